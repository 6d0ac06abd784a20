"""The FDK filter's FFT schedule, restated on the CPU: consecutive radix-2
stages of an in-place DIF forward / DIT inverse transform (natural order in,
bit-reversed spectrum, natural order out) fused into radix-8 passes with a
radix-4 or radix-2 remainder, with the same butterflies and twiddle indices
as the kernel.  The fused schedule must give exactly the radix-2 result
(same operations in the same order), and that result must equal the
zero-padded circular convolution computed with numpy's FFT."""
import numpy as np
import pytest


def _tw(L):
    return np.exp(-2j * np.pi * np.arange(max(L // 2, 1)) / L)


def _radix2(x, H, tw):
    b = x.copy()
    L = len(b)
    span, ts = L // 2, 1
    while span >= 1:
        for t in range(L // 2):
            j = t & (span - 1)
            i0 = ((t - j) << 1) + j
            u, w = b[i0], b[i0 + span]
            b[i0], b[i0 + span] = u + w, (u - w) * tw[j * ts]
        span, ts = span >> 1, ts << 1
    b *= H
    span, ts = 1, L // 2
    while span < L:
        for t in range(L // 2):
            j = t & (span - 1)
            i0 = ((t - j) << 1) + j
            w = b[i0 + span] * np.conj(tw[j * ts])
            u = b[i0]
            b[i0], b[i0 + span] = u + w, u - w
        span, ts = span << 1, ts >> 1
    return b


def _fused(x, H, tw):
    b = x.copy()
    L = len(b)
    logL = L.bit_length() - 1
    span, rem = L // 2, logL
    while rem >= 3:                                   # radix-8 DIF: stages S, S/2, S/4
        E, ts1 = span >> 2, L // (2 * span)
        for t in range(L // 8):
            j = t & (E - 1)
            i0 = ((t - j) << 3) + j
            x8 = [b[i0 + k * E] for k in range(8)]
            y = [0j] * 8
            for k in range(4):
                y[k] = x8[k] + x8[k + 4]
                y[k + 4] = (x8[k] - x8[k + 4]) * tw[(j + k * E) * ts1]
            c0, c1, c3 = tw[j * 2 * ts1], tw[(j + E) * 2 * ts1], tw[j * 4 * ts1]
            for q in (0, 4):
                z0, z2 = y[q] + y[q + 2], (y[q] - y[q + 2]) * c0
                z1, z3 = y[q + 1] + y[q + 3], (y[q + 1] - y[q + 3]) * c1
                b[i0 + q * E], b[i0 + (q + 1) * E] = z0 + z1, (z0 - z1) * c3
                b[i0 + (q + 2) * E], b[i0 + (q + 3) * E] = z2 + z3, (z2 - z3) * c3
        span, rem = span >> 3, rem - 3
    if rem == 2:                                      # radix-4 DIF: stages S, S/2
        Q, ts = span >> 1, L // (2 * span)
        for t in range(L // 4):
            j = t & (Q - 1)
            i0 = ((t - j) << 2) + j
            x0, x1, x2, x3 = b[i0], b[i0 + Q], b[i0 + span], b[i0 + span + Q]
            y0, y2 = x0 + x2, (x0 - x2) * tw[j * ts]
            y1, y3 = x1 + x3, (x1 - x3) * tw[(j + Q) * ts]
            c = tw[j * 2 * ts]
            b[i0], b[i0 + Q], b[i0 + span], b[i0 + span + Q] = y0 + y1, (y0 - y1) * c, y2 + y3, (y2 - y3) * c
    elif rem == 1:
        for t in range(L // 2):
            u, w = b[2 * t], b[2 * t + 1]
            b[2 * t], b[2 * t + 1] = u + w, (u - w) * tw[0]
    b *= H
    span, rem = 1, logL % 3
    if rem == 1:
        for t in range(L // 2):
            w = b[2 * t + 1] * np.conj(tw[0])
            u = b[2 * t]
            b[2 * t], b[2 * t + 1] = u + w, u - w
        span = 2
    elif rem == 2:                                    # radix-4 DIT: stages 1, 2
        for t in range(L // 4):
            i0 = 4 * t
            c1, ca, cb = np.conj(tw[0]), np.conj(tw[0]), np.conj(tw[L // 4])
            x0, x1, x2, x3 = b[i0], b[i0 + 1], b[i0 + 2], b[i0 + 3]
            w1, w3 = x1 * c1, x3 * c1
            y0, y1, y2, y3 = x0 + w1, x0 - w1, x2 + w3, x2 - w3
            wa, wb = y2 * ca, y3 * cb
            b[i0], b[i0 + 2], b[i0 + 1], b[i0 + 3] = y0 + wa, y0 - wa, y1 + wb, y1 - wb
        span = 4
    while span < L:                                   # radix-8 DIT: stages S, 2S, 4S
        ts1 = L // (2 * span)
        for t in range(L // 8):
            j = t & (span - 1)
            i0 = ((t - j) << 3) + j
            x8 = [b[i0 + k * span] for k in range(8)]
            c1 = np.conj(tw[j * ts1])
            y = [0j] * 8
            for k in (0, 2, 4, 6):
                w = x8[k + 1] * c1
                y[k], y[k + 1] = x8[k] + w, x8[k] - w
            ca, cb = np.conj(tw[j * (ts1 >> 1)]), np.conj(tw[(j + span) * (ts1 >> 1)])
            z = [0j] * 8
            for q in (0, 4):
                wa, wb = y[q + 2] * ca, y[q + 3] * cb
                z[q], z[q + 2], z[q + 1], z[q + 3] = y[q] + wa, y[q] - wa, y[q + 1] + wb, y[q + 1] - wb
            for k in range(4):
                w = z[k + 4] * np.conj(tw[(j + k * span) * (ts1 >> 2)])
                b[i0 + k * span], b[i0 + (k + 4) * span] = z[k] + w, z[k] - w
        span <<= 3
    return b


@pytest.mark.parametrize("logL", range(1, 10))
def test_fused_schedule_equals_radix2_and_the_convolution(logL):
    L = 1 << logL
    rng = np.random.default_rng(logL)
    x = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    H = rng.standard_normal(L)                       # response in bit-reversed order
    tw = _tw(L)
    r2 = _radix2(x, H, tw)
    assert np.array_equal(_fused(x, H, tw), r2)
    rev = np.array([int(format(i, f"0{logL}b")[::-1], 2) for i in range(L)])
    Hn = np.empty(L)
    Hn[rev] = H
    want = np.fft.ifft(Hn * np.fft.fft(x)) * L
    assert np.max(np.abs(r2 - want)) < 1e-12 * L * np.max(np.abs(want))
