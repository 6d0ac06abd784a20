"""What the trained network gains over the method without it (the learned
prior inside the Krylov solver of section 2.2.1): a U-Net trained on the
GPU by the library's own kernels, on sparse-view vs dense-view CGLS pairs
that the library's projectors generate, lets PnP-CGLS reach a PSNR that
plain CGLS does not reach in the same number of iterations on a held-out
phantom.  Every PSNR here is judged by the FP64 oracle on the saved
iterates (x_gt = the phantom, over the FOV cylinder).

A small instance of the sparse-view workload: 64^3 at 1 mm, 20 sparse and
160 dense views, 96 x 96 detector at 1.6 mm, textured random-ellipsoid
phantoms (training seeds 0..11, held-out seed 100), 1500 Adam steps on
32^3 crops.  Two gains are checked: the trained network alone lifts every
CGLS iterate it was trained on (k = 5, 10, 15, 20) by more than 1 dB on the
held-out phantom, and inside PnP-CGLS at least one proposal passes the 5 %
residual test and the best iterate beats plain CGLS's best by more than
1 dB (on this instance the first proposal's residual ratio is near 0.85
and both gains are 3-4 dB)."""
import numpy as np
import pytest

import synth
from synth import Geometry

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

GEO = Geometry(DSD=1536.0, DSO=1000.0, nVoxel=(64, 64, 64), dVoxel=(1.0, 1.0, 1.0), nDetector=(96, 96),
               dDetector=(1.6, 1.6))
NITER = 30


@pytest.fixture(scope="module")
def P():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2412_10129_amd as P
    return P


def test_trained_prior_beats_plain_cgls(P, orc):
    from paper_2412_10129_amd import learned as LN
    plan = P.Plan(GEO, synth.circular_angles(20))
    dense = P.Plan(GEO, synth.circular_angles(160))
    vols = [synth.textured_phantom(GEO, s) for s in range(12)]
    inputs, targets = LN.make_pairs(plan, dense, vols)
    net = P.UNet(seed=0)
    mse = LN.train(net, inputs, targets, steps=1500, crop=32, batch=4, seed=0, log_every=375, log=lambda m: None)
    assert mse[-1] < mse[0]
    del inputs, targets

    x_gt = synth.textured_phantom(GEO, 100)
    xg = torch.from_numpy(x_gt).cuda()
    b = plan.forward(xg, kind="interp")
    mask = orc.fov_mask(GEO)
    # the network on its own: denoised CGLS-k iterates against the iterates
    _, h = P.cgls(plan, b, 20, kind="interp", snapshots=LN.KS)
    for k in LN.KS:
        xk = h["snapshots"][k]
        before = orc.psnr(xk.cpu().numpy(), x_gt, mask)
        after = orc.psnr(net.forward(xk).cpu().numpy(), x_gt, mask)
        assert after > before + 1.0, (k, before, after)
    best = {}
    for name, every in (("cgls", NITER + 1), ("pnp", 5)):
        its = []
        _, h = P.pnp_cgls(plan, b, NITER, net, every=every, kind="interp", keep=its)
        judged = [orc.psnr(x.cpu().numpy(), x_gt, mask) for x in its]
        best[name] = (max(judged), h.get("accepted"))
    assert any(best["pnp"][1]), best            # at least one proposal passed the residual test
    assert best["pnp"][0] > best["cgls"][0] + 1.0, best
