// C entry points of the learned-prior kernels (declared in ctmi_unet.h): argument
// checks, then the launchers in unet.hip.  Every check happens before
// anything is enqueued, so a failing call has no effect.
#include <cmath>
#include <cstdarg>

#include "ctmi_internal.h"

using ctmi::api_fail;
using ctmi::api_hip;

namespace {

int ok_or(hipError_t e, const char* what) { return e == hipSuccess ? CTMI_OK : api_hip(e, what); }

int check_dims(int n, int d, int h, int w)
{
    if (n < 0 || d < 0 || h < 0 || w < 0) return api_fail(CTMI_EINVAL, "negative tensor size");
    if (n > 65535 || d > 65535 * 2) return api_fail(CTMI_EOVERFLOW, "batch above 65535 or depth above 131070");
    const int64_t tiles = ((int64_t)w / 16 + 1) * ((int64_t)h / 8 + 1) * ((int64_t)d / 2 + 1) * (int64_t)n;
    if (tiles >= ((int64_t)1 << 31)) return api_fail(CTMI_EOVERFLOW, "volume too large for the tile index range");
    return CTMI_OK;
}

bool empty(int n, int d, int h, int w) { return n == 0 || d == 0 || h == 0 || w == 0; }

int check_tensor(const void* p, int c, int ld, int cmul, const char* name)
{
    if (!p) return api_fail(CTMI_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return api_fail(CTMI_EINVAL, "%s is not 16-byte aligned", name);
    if (c <= 0 || c % cmul != 0) return api_fail(CTMI_EINVAL, "%s: %d channels is not a positive multiple of %d", name, c, cmul);
    if (ld < c || ld % 8 != 0) return api_fail(CTMI_EINVAL, "%s: row length %d must be >= %d and a multiple of 8", name, ld, c);
    return CTMI_OK;
}

int check_cout(int cout)
{
    if (cout != 16 && cout != 32 && cout != 64 && cout != 128)
        return api_fail(CTMI_EUNSUPPORTED, "output channels %d: 16, 32, 64 or 128 supported", cout);
    return CTMI_OK;
}

int check_ptr4(const void* p, const char* name)
{
    if (!p) return api_fail(CTMI_EINVAL, "%s is NULL", name);
    if (reinterpret_cast<uintptr_t>(p) % 4 != 0) return api_fail(CTMI_EINVAL, "%s is not 4-byte aligned", name);
    return CTMI_OK;
}

int check_ws(const void* ws, size_t have, size_t need)
{
    if (!ws) return api_fail(CTMI_EWORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(ws) % 16 != 0) return api_fail(CTMI_EINVAL, "workspace is not 16-byte aligned");
    if (have < need) return api_fail(CTMI_EWORKSPACE, "workspace of %zu bytes is below the %zu required", have, need);
    return CTMI_OK;
}

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

}  // namespace

extern "C" {

int ctmi_conv3d_bf16_fwd(int n, int d, int h, int w, const uint16_t* in0, int c0, int ld0, const uint16_t* in1,
                         int c1, int ld1, const uint16_t* wt, const float* bias, int cout, int relu, uint16_t* out,
                         int ldo, void* stream)
{
    int rc;
    if ((rc = check_dims(n, d, h, w)) || (rc = check_cout(cout)) || (rc = check_tensor(in0, c0, ld0, 16, "in0")) ||
        (rc = check_tensor(out, cout, ldo, 16, "out")))
        return rc;
    if (c1 != 0 && (rc = check_tensor(in1, c1, ld1, 16, "in1"))) return rc;
    if (c0 + c1 > 1024) return api_fail(CTMI_EUNSUPPORTED, "more than 1024 input channels");
    if (!wt || reinterpret_cast<uintptr_t>(wt) % 16 != 0) return api_fail(CTMI_EINVAL, "weights NULL or not 16-byte aligned");
    if (bias && (rc = check_ptr4(bias, "bias"))) return rc;
    if (empty(n, d, h, w)) return CTMI_OK;
    ctmi::UnetConv3 a{in0, c0, ld0, c1 ? in1 : nullptr, c1, c1 ? ld1 : 8, wt, bias, nullptr, 0, out, ldo,
                      cout, relu ? 1 : 0, n, d, h, w};
    return ok_or(ctmi::launch_unet_conv3(a, S(stream)), "conv3d_bf16_fwd");
}

int ctmi_conv3d_bf16_dgrad(int n, int d, int h, int w, const uint16_t* dz, int cout, int ldz, const uint16_t* wd,
                           int cin, const uint16_t* mask, int ldm, uint16_t* dx, int ldx, void* stream)
{
    int rc;
    if ((rc = check_dims(n, d, h, w)) || (rc = check_cout(cin)) || (rc = check_tensor(dz, cout, ldz, 16, "dz")) ||
        (rc = check_tensor(dx, cin, ldx, 16, "dx")))
        return rc;
    if (cout > 1024) return api_fail(CTMI_EUNSUPPORTED, "more than 1024 output channels");
    if (mask && (rc = check_tensor(mask, cin, ldm, 16, "mask"))) return rc;
    if (!wd || reinterpret_cast<uintptr_t>(wd) % 16 != 0) return api_fail(CTMI_EINVAL, "weights NULL or not 16-byte aligned");
    if (empty(n, d, h, w)) return CTMI_OK;
    ctmi::UnetConv3 a{dz, cout, ldz, nullptr, 0, 8, wd, nullptr, mask, mask ? ldm : 0, dx, ldx, cin, 0, n, d, h, w};
    return ok_or(ctmi::launch_unet_conv3(a, S(stream)), "conv3d_bf16_dgrad");
}

size_t ctmi_conv3d_wgrad_workspace_bytes(int n, int d, int h, int w, int cin, int cout)
{
    if (n <= 0 || d <= 0 || h <= 0 || w <= 0 || cin <= 0 || cout <= 0) return 0;
    return ctmi::unet_wgrad_ws_bytes(n, d, h, w, cin, cout);
}

int ctmi_conv3d_bf16_wgrad(int n, int d, int h, int w, const uint16_t* in0, int c0, int ld0, const uint16_t* in1,
                           int c1, int ld1, const uint16_t* dz, int cout, int ldz, float* dw, float* db,
                           int accumulate, void* ws, size_t ws_bytes, void* stream)
{
    int rc;
    if ((rc = check_dims(n, d, h, w)) || (rc = check_cout(cout)) || (rc = check_tensor(in0, c0, ld0, 16, "in0")) ||
        (rc = check_tensor(dz, cout, ldz, 16, "dz")) || (rc = check_ptr4(dw, "dw")))
        return rc;
    if (c1 != 0 && (rc = check_tensor(in1, c1, ld1, 16, "in1"))) return rc;
    if (db && (rc = check_ptr4(db, "db"))) return rc;
    if (empty(n, d, h, w)) return CTMI_OK;
    if ((rc = check_ws(ws, ws_bytes, ctmi::unet_wgrad_ws_bytes(n, d, h, w, c0 + c1, cout)))) return rc;
    ctmi::UnetWgrad a{in0, c0, ld0, c1 ? in1 : nullptr, c1, c1 ? ld1 : 8, dz, ldz, cout, n, d, h, w,
                      static_cast<float*>(ws)};
    return ok_or(ctmi::launch_unet_conv3_wgrad(a, dw, db, accumulate ? 1 : 0, S(stream)), "conv3d_bf16_wgrad");
}

int ctmi_conv3d_pack_weights(const float* w, int cout, int cin, uint16_t* wf, uint16_t* wd, void* stream)
{
    int rc;
    if ((rc = check_ptr4(w, "w"))) return rc;
    if (cout <= 0 || cin <= 0) return api_fail(CTMI_EINVAL, "channel counts must be positive");
    if (!wf) return api_fail(CTMI_EINVAL, "wf is NULL");
    return ok_or(ctmi::launch_unet_pack_conv3(w, cout, cin, wf, wd, S(stream)), "conv3d_pack_weights");
}

int ctmi_unet_pack_input(const float* x, int64_t nvox, uint16_t* out, void* stream)
{
    int rc;
    if ((rc = check_ptr4(x, "x"))) return rc;
    if (nvox < 0) return api_fail(CTMI_EINVAL, "negative length");
    if (!out || reinterpret_cast<uintptr_t>(out) % 16 != 0) return api_fail(CTMI_EINVAL, "out NULL or not 16-byte aligned");
    if (nvox == 0) return CTMI_OK;
    return ok_or(ctmi::launch_unet_pack_input(x, nvox, out, S(stream)), "unet_pack_input");
}

int ctmi_pool2(int n, int d, int h, int w, int c, const uint16_t* in, int ldi, uint16_t* out, int ldo, void* stream)
{
    int rc;
    if ((rc = check_dims(n, 2 * d, 2 * h, 2 * w)) || (rc = check_tensor(in, c, ldi, 8, "in")) ||
        (rc = check_tensor(out, c, ldo, 8, "out")))
        return rc;
    if (empty(n, d, h, w)) return CTMI_OK;
    return ok_or(ctmi::launch_unet_pool2(in, ldi, n, d, h, w, c, out, ldo, S(stream)), "pool2");
}

int ctmi_pool2_skip_grad(int n, int d, int h, int w, int c, const uint16_t* e, int lde, const uint16_t* dp, int ldp,
                         const uint16_t* dcat, int ldc, uint16_t* out, int ldo, void* stream)
{
    int rc;
    if ((rc = check_dims(n, d, h, w)) || (rc = check_tensor(e, c, lde, 8, "e")) ||
        (rc = check_tensor(dp, c, ldp, 8, "dp")) || (rc = check_tensor(dcat, c, ldc, 8, "dcat")) ||
        (rc = check_tensor(out, c, ldo, 8, "out")))
        return rc;
    if (d % 2 || h % 2 || w % 2) return api_fail(CTMI_EINVAL, "fine-grid sizes must be even");
    if (empty(n, d, h, w)) return CTMI_OK;
    return ok_or(ctmi::launch_unet_skip_grad(e, lde, dp, ldp, dcat, ldc, n, d, h, w, c, out, ldo, S(stream)),
                 "pool2_skip_grad");
}

int ctmi_upsample2(int n, int d, int h, int w, const uint16_t* x, int cin, int ldx, const uint16_t* wt,
                   const float* bias, int cout, uint16_t* out, int ldo, void* stream)
{
    int rc;
    if ((rc = check_dims(n, 2 * d, 2 * h, 2 * w)) || (rc = check_tensor(x, cin, ldx, 8, "x")) ||
        (rc = check_tensor(out, cout, ldo, 8, "out")) || (rc = check_tensor(wt, cin, cin, 8, "weights")))
        return rc;
    if (bias && (rc = check_ptr4(bias, "bias"))) return rc;
    if (empty(n, d, h, w)) return CTMI_OK;
    return ok_or(ctmi::launch_unet_up2(x, ldx, cin, wt, bias, cout, n, d, h, w, out, ldo, S(stream)), "upsample2");
}

int ctmi_upsample2_dgrad(int n, int d, int h, int w, const uint16_t* g, int cout, int ldg, const uint16_t* wt, int cin,
                         const uint16_t* below, int ldb, uint16_t* dx, int ldx, void* stream)
{
    int rc;
    if ((rc = check_dims(n, 2 * d, 2 * h, 2 * w)) || (rc = check_tensor(g, cout, ldg, 8, "g")) ||
        (rc = check_tensor(dx, cin, ldx, 8, "dx")) || (rc = check_tensor(wt, cin, cin, 8, "weights")))
        return rc;
    if (below && (rc = check_tensor(below, cin, ldb, 8, "below"))) return rc;
    if (empty(n, d, h, w)) return CTMI_OK;
    return ok_or(ctmi::launch_unet_up2_dgrad(g, ldg, cout, wt, cin, below, ldb, n, d, h, w, dx, ldx, S(stream)),
                 "upsample2_dgrad");
}

size_t ctmi_upsample2_wgrad_workspace_bytes(int n, int d, int h, int w, int cin, int cout)
{
    if (n <= 0 || d <= 0 || h <= 0 || w <= 0 || cin <= 0 || cout <= 0) return 0;
    return ctmi::unet_up2_wgrad_ws_bytes(n, d, h, w, cin, cout);
}

int ctmi_upsample2_wgrad(int n, int d, int h, int w, const uint16_t* x, int cin, int ldx, const uint16_t* g, int cout,
                         int ldg, float* dw, float* db, int accumulate, void* ws, size_t ws_bytes, void* stream)
{
    int rc;
    if ((rc = check_dims(n, 2 * d, 2 * h, 2 * w)) || (rc = check_tensor(x, cin, ldx, 16, "x")) ||
        (rc = check_tensor(g, cout, ldg, 16, "g")) || (rc = check_ptr4(dw, "dw")))
        return rc;
    if (db && (rc = check_ptr4(db, "db"))) return rc;
    if (empty(n, d, h, w)) return CTMI_OK;
    if ((rc = check_ws(ws, ws_bytes, ctmi::unet_up2_wgrad_ws_bytes(n, d, h, w, cin, cout)))) return rc;
    return ok_or(ctmi::launch_unet_up2_wgrad(x, ldx, cin, g, ldg, cout, n, d, h, w, static_cast<float*>(ws), dw, db,
                                             accumulate ? 1 : 0, S(stream)),
                 "upsample2_wgrad");
}

int ctmi_unet_head(int64_t nvox, const float* xin, const uint16_t* act, int c, int lda, const uint16_t* hw,
                   const float* hb, float* out, void* stream)
{
    int rc;
    if (nvox < 0) return api_fail(CTMI_EINVAL, "negative length");
    if ((rc = check_ptr4(xin, "x_in")) || (rc = check_tensor(act, c, lda, 8, "act")) || (rc = check_ptr4(out, "out")) ||
        (rc = check_ptr4(hb, "hb")))
        return rc;
    if (!hw) return api_fail(CTMI_EINVAL, "hw is NULL");
    if (nvox == 0) return CTMI_OK;
    return ok_or(ctmi::launch_unet_head(xin, act, lda, c, hw, hb, nvox, out, S(stream)), "unet_head");
}

size_t ctmi_unet_head_workspace_bytes(void) { return ctmi::unet_head_ws_bytes(); }

int ctmi_unet_head_mse_bwd(int64_t nvox, const float* out, const float* target, const uint16_t* act, int lda,
                           const uint16_t* hw, uint16_t* dz, int ldz, double* sums, float* dhead, void* ws,
                           size_t ws_bytes, void* stream)
{
    int rc;
    if (nvox <= 0) return api_fail(CTMI_EINVAL, "the loss needs at least one voxel");
    if ((rc = check_ptr4(out, "out")) || (rc = check_ptr4(target, "target")) ||
        (rc = check_tensor(act, 16, lda, 8, "act")) || (rc = check_tensor(dz, 16, ldz, 8, "dz")))
        return rc;
    if (!hw) return api_fail(CTMI_EINVAL, "hw is NULL");
    if (!sums || reinterpret_cast<uintptr_t>(sums) % 8 != 0) return api_fail(CTMI_EINVAL, "sums NULL or not 8-byte aligned");
    if (dhead && (rc = check_ptr4(dhead, "dhead"))) return rc;
    if ((rc = check_ws(ws, ws_bytes, ctmi::unet_head_ws_bytes()))) return rc;
    return ok_or(ctmi::launch_unet_head_loss_bwd(out, target, act, lda, hw, nvox, dz, ldz, static_cast<double*>(ws),
                                                 sums, dhead, S(stream)),
                 "unet_head_mse_bwd");
}

int ctmi_adam_step(float* w, float* m, float* v, const float* g, int64_t n, float lr, float beta1, float beta2,
                   float eps, int64_t t, void* stream)
{
    int rc;
    if ((rc = check_ptr4(w, "w")) || (rc = check_ptr4(m, "m")) || (rc = check_ptr4(v, "v")) || (rc = check_ptr4(g, "g")))
        return rc;
    if (n < 0 || t < 1) return api_fail(CTMI_EINVAL, "negative length or step count below 1");
    if (!(beta1 >= 0.0f && beta1 < 1.0f && beta2 >= 0.0f && beta2 < 1.0f && eps > 0.0f))
        return api_fail(CTMI_EINVAL, "Adam needs 0 <= beta < 1 and eps > 0");
    if (n == 0) return CTMI_OK;
    const double bc1 = 1.0 - std::pow((double)beta1, (double)t);
    const double bc2 = 1.0 - std::pow((double)beta2, (double)t);
    return ok_or(ctmi::launch_unet_adam(w, m, v, g, n, beta1, beta2, (float)(lr / bc1), (float)(1.0 / std::sqrt(bc2)), eps,
                                        S(stream)),
                 "adam_step");
}

int ctmi_to_bf16(const float* a, int64_t n, uint16_t* out, void* stream)
{
    int rc;
    if ((rc = check_ptr4(a, "a"))) return rc;
    if (!out || n < 0) return api_fail(CTMI_EINVAL, "out NULL or negative length");
    if (n == 0) return CTMI_OK;
    return ok_or(ctmi::launch_unet_to_bf16(a, n, out, S(stream)), "to_bf16");
}

}  // extern "C"
