// Internal declarations of libctmi: the device view table, the ray helpers
// that the forward projectors and their transposes share, and the kernel
// launchers.  The forward and adjoint kernels include the same inline
// helpers so that both evaluate every matrix entry with identical FP32
// arithmetic (explicit fmaf, no contraction), which makes the adjoint exact
// up to summation order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "../../include/ctmi.h"

namespace ctmi {

// Per-view geometry, 32 floats (128 B, one cache line) per view.
//   S      source, voxel-cell coordinates (volume corner 0, one unit per voxel)
//   P00    centre of detector pixel (0, 0), same coordinates
//   DU/DV  step per pixel index along u / v, same coordinates
//   MU/MV/MW rows of the 3x4 matrix taking voxel-centre indices (ix,iy,iz,1)
//          to (fu W, fv W, W), W = U / DSO, (fu, fv) pixel-index coordinates
struct ViewGeo {
    float S[3];
    float P00[3];
    float DU[3];
    float DV[3];
    float MU[4];
    float MV[4];
    float MW[4];
    float pad[8];
};
static_assert(sizeof(ViewGeo) == 128, "view table row must be 128 bytes");

// The same geometry in FP64 (source, pixel (0,0) centre, pixel steps, in
// voxel-cell coordinates) for the once-per-ray setup: the source lies
// thousands of voxels from the volume, and FP32 positions that far out carry
// errors of ~1e-4 voxel, so rays are set up in FP64 and re-anchored next to
// the volume before the FP32 per-sample loops.
struct ViewGeo64 {
    double S[3];
    double P00[3];
    double DU[3];
    double DV[3];
    double pad[4];
};
static_assert(sizeof(ViewGeo64) == 128, "FP64 view table row must be 128 bytes");

// Voxel bricks of the matched adjoints (x, y, z extents) and the cells in
// the upper shell of one brick (faces x, y, z) that the interpolated adjoint
// hands to its neighbours.
#ifndef CTMI_BWD_BX
#define CTMI_BWD_BX 16
#endif
#ifndef CTMI_BWD_BY
#define CTMI_BWD_BY 16
#endif
#ifndef CTMI_BWD_BZ
#define CTMI_BWD_BZ 8
#endif
#define CTMI_HALO_SLOTS \
    ((CTMI_BWD_BY + 1) * (CTMI_BWD_BZ + 1) + CTMI_BWD_BX * (CTMI_BWD_BZ + 1) + CTMI_BWD_BX * CTMI_BWD_BY)

struct VolDims {
    int nx, ny, nz;
    float hx, hy, hz;  // voxel size, mm
};

struct DetDims {
    int nu, nv;
};

// Everything a plan holds.
struct Plan {
    ctmi_geometry geo;
    int64_t nviews;
    bool circular;        // every view is the circular default (FDK is defined for it)
    int device;
    ViewGeo* d_views;     // [nviews]
    ViewGeo64* d_views64; // [nviews]
    float* d_filter;      // [fft_len] Ram-Lak response, bit-reversed order, 1/L folded in
    float2* d_twiddle;    // [fft_len / 2] exp(-2 pi i k / L)
    int fft_len;
    int fft_log2;
    VolDims vol;
    DetDims det;
    float ds;             // interpolated-projector step, mm
    float entry_siddon;   // largest single adjoint term factor, Siddon (one chord, mm)
    float round_interp;   // most one ray adds to one adjoint cell per unit y: K ds (mm)
    float round_siddon;   // the same for Siddon: one chord (mm)
};

// Voxel bricks of the matched adjoints along each axis, and the bytes of the
// interpolated adjoint's workspace (CTMI_HALO_SLOTS floats per brick).
int64_t adjoint_bricks(const Plan& p);
size_t interp_adjoint_ws_bytes(const Plan& p);

// ------------------------------------------------------------ launchers
hipError_t launch_forward_siddon(const Plan& p, const float* vol, float* proj, int64_t view0, int64_t nviews,
                                 hipStream_t s);
hipError_t launch_forward_interp(const Plan& p, const float* vol, float* proj, int64_t view0, int64_t nviews,
                                 hipStream_t s);
hipError_t launch_backward_siddon(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                                  float beta, hipStream_t s);
hipError_t launch_backward_interp(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                                  float beta, float* shell, hipStream_t s);
hipError_t launch_backward_fdk(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                               float beta, hipStream_t s);
hipError_t launch_fdk_filter(const Plan& p, int wang, const float* proj, float* out, int64_t view0,
                             int64_t nviews, hipStream_t s);

// reductions / vector ops
int reduce_blocks(int64_t n);
hipError_t launch_dot(const float* a, const float* b, int64_t n, double* out, double* ws, hipStream_t s);
hipError_t launch_axpby(int64_t n, float a, const float* x, float b, float* y, hipStream_t s);
hipError_t launch_cgls_xr(float* x, const float* p, int64_t nvol, float* r, const float* q, int64_t nproj,
                          const double* gamma, const double* delta, double* rnorm2, double* ws, hipStream_t s);
hipError_t launch_cgls_p(float* p, const float* s_, int64_t n, const double* g0, const double* g1, hipStream_t s);
hipError_t launch_recip(const float* in, float* out, int64_t n, hipStream_t s);
hipError_t launch_sart_residual(const float* b, const float* ax, const float* w, float* out, int64_t n,
                                hipStream_t s);
hipError_t launch_sart_update(float* x, const float* v, const float* bp, int64_t n, float lam, int nonneg,
                              hipStream_t s);
hipError_t launch_em_ratio(const float* b, const float* ax, float* out, int64_t n, hipStream_t s);
hipError_t launch_awtv_grad(const float* x, float* g, int nz, int ny, int nx, float delta, float eps, hipStream_t s);
hipError_t launch_tv_step(float* x, const float* g, int64_t n, const double* gnorm2, float step, hipStream_t s);
hipError_t launch_em_update(float* x, const float* v, const float* bp, int64_t n, hipStream_t s);
hipError_t launch_fov_sq_err(const Plan& p, const float* x, const float* gt, double* out, double* ws,
                             hipStream_t s);

// ---------------------------------------------------------------- U-Net
// Argument block of the 3x3x3 BF16 convolution (forward, and data gradient
// with flipped weights).  Tensors are channels-last [n][d][h][w][ld].
struct UnetConv3 {
    const uint16_t* in0;
    int c0, ld0;            // input channels [0, c0) from in0
    const uint16_t* in1;
    int c1, ld1;            // input channels [c0, c0 + c1) from in1 (c1 may be 0)
    const uint16_t* wt;     // [cout][27][c0 + c1] BF16
    const float* bias;      // [cout] or null
    const uint16_t* mask;   // output multiplied by (mask > 0) when not null
    int ldm;
    uint16_t* out;
    int ldo;
    int cout, relu;
    int n, d, h, w;
};

struct UnetWgrad {
    const uint16_t* in0;
    int c0, ld0;
    const uint16_t* in1;
    int c1, ld1;
    const uint16_t* dz;     // output gradient [..][ldz], channels [0, cout)
    int ldz;
    int cout;
    int n, d, h, w;
    float* partial;         // workspace
};

hipError_t launch_unet_conv3(const UnetConv3& a, hipStream_t s);
int unet_wgrad_splits(int n, int d, int h, int w, int cin, int cout);
size_t unet_wgrad_ws_bytes(int n, int d, int h, int w, int cin, int cout);
hipError_t launch_unet_conv3_wgrad(const UnetWgrad& a, float* dw, float* db, int accumulate, hipStream_t s);
hipError_t launch_unet_pack_input(const float* x, int64_t nvox, uint16_t* out, hipStream_t s);
hipError_t launch_unet_pool2(const uint16_t* in, int ldi, int n, int d, int h, int w, int c, uint16_t* out, int ldo,
                             hipStream_t s);
hipError_t launch_unet_skip_grad(const uint16_t* e, int lde, const uint16_t* dp, int ldp, const uint16_t* dcat,
                                 int ldc, int n, int d, int h, int w, int c, uint16_t* out, int ldo, hipStream_t s);
hipError_t launch_unet_up2(const uint16_t* x, int ldx, int cin, const uint16_t* wt, const float* bias, int cout,
                           int n, int d, int h, int w, uint16_t* out, int ldo, hipStream_t s);
hipError_t launch_unet_up2_dgrad(const uint16_t* g, int ldg, int cout, const uint16_t* wt, int cin,
                                 const uint16_t* below, int ldb, int n, int d, int h, int w, uint16_t* out, int ldo,
                                 hipStream_t s);
size_t unet_up2_wgrad_ws_bytes(int n, int d, int h, int w, int cin, int cout);
hipError_t launch_unet_up2_wgrad(const uint16_t* x, int ldx, int cin, const uint16_t* g, int ldg, int cout, int n,
                                 int d, int h, int w, float* ws, float* dw, float* db, int accumulate, hipStream_t s);
hipError_t launch_unet_head(const float* xin, const uint16_t* act, int lda, int c, const uint16_t* hw,
                            const float* hb, int64_t nvox, float* out, hipStream_t s);
size_t unet_head_ws_bytes();
hipError_t launch_unet_head_loss_bwd(const float* out, const float* tgt, const uint16_t* act, int lda,
                                     const uint16_t* hw, int64_t nvox, uint16_t* dz, int ldz, double* ws,
                                     double* sums, float* dhead, hipStream_t s);
hipError_t launch_unet_adam(float* w, float* m, float* v, const float* g, int64_t n, float b1, float b2, float lr_t,
                            float inv_sqrt_bc2, float eps, hipStream_t s);
hipError_t launch_unet_pack_conv3(const float* w, int cout, int cin, uint16_t* wf, uint16_t* wd, hipStream_t s);
hipError_t launch_unet_to_bf16(const float* a, int64_t n, uint16_t* out, hipStream_t s);

// curved detectors: flat (plan) and curved pixel grids, mm
struct FlatDet {
    int nu, nv;
    double du, dv, ou, ov;
};
struct CurvedDet {
    int nu, nv;
    double du, dv, ou, ov;  // du, ou along the arc
    double R;               // arc radius
};
hipError_t launch_flatten_curved(const Plan& p, const CurvedDet& c, const float* curved, float* flat, int64_t nviews,
                                 hipStream_t s);

// measurement ceilings
hipError_t launch_stream_copy(const float* src, float* dst, int64_t n, hipStream_t s);
int fma_loop_chains();
hipError_t launch_fma_loop(float* out, int blocks, int iters, hipStream_t s);

// backprojection entry points: argument checks (all but the workspace) and
// the launch with a checked workspace
int check_backproject(const ctmi_plan* plan, int bp, const float* proj, float* vol, int64_t view0, int64_t nviews,
                      float beta);
int run_backproject(const ctmi_plan* plan, int bp, const float* proj, float* vol, int64_t view0, int64_t nviews,
                    float beta, float* ws, void* stream);

// error reporting shared by the entry points (thread-local message)
int api_fail(int code, const char* fmt, ...);
int api_hip(hipError_t e, const char* what);


#ifdef __HIPCC__
// ------------------------------------------------------------------------
// Device helpers shared by the forward kernels and their transposes.
// ------------------------------------------------------------------------
#define CTMI_INF __builtin_huge_valf()

// Ray from the source to the centre of pixel (iu, iv), voxel-cell coordinates.
__device__ __forceinline__ void pixel_ray(const ViewGeo& g, int iu, int iv, float S[3], float d[3])
{
    const float fu = (float)iu, fv = (float)iv;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        S[a] = g.S[a];
        const float P = __builtin_fmaf(fv, g.DV[a], __builtin_fmaf(fu, g.DU[a], g.P00[a]));
        d[a] = P - S[a];
    }
}

// World length (mm) of the direction vector d given in voxel units.
__device__ __forceinline__ float world_length(const float d[3], const VolDims& v)
{
    const float x = d[0] * v.hx, y = d[1] * v.hy, z = d[2] * v.hz;
    return __builtin_sqrtf(__builtin_fmaf(x, x, __builtin_fmaf(y, y, z * z)));
}

// --- Siddon ---------------------------------------------------------------
// Crossing parameter of plane q on an axis: alpha = q * inv + c, c = -S inv.
struct SiddonAxis {
    float inv, c;
    int step;  // +1, -1 or 0 (ray parallel to the planes)
};

__device__ __forceinline__ SiddonAxis siddon_axis(float S, float d)
{
    SiddonAxis ax;
    if (d != 0.0f) {
        // the hardware reciprocal (1 ulp): every kernel forms its crossing
        // parameters from this same value
        ax.inv = __builtin_amdgcn_rcpf(d);
        ax.c = -S * ax.inv;
        ax.step = d > 0.0f ? 1 : -1;
    } else {
        ax.inv = 0.0f;
        ax.c = CTMI_INF;
        ax.step = 0;
    }
    return ax;
}

__device__ __forceinline__ float plane_alpha(const SiddonAxis& ax, float q)
{
    return ax.step ? __builtin_fmaf(q, ax.inv, ax.c) : CTMI_INF;
}

// Clip alpha to the slab [lo, hi] of one axis (lo, hi plane coordinates).
// Returns false when a parallel ray lies outside the slab.
__device__ __forceinline__ bool slab_clip(const SiddonAxis& ax, float S, float lo, float hi, float& amin,
                                          float& amax)
{
    if (ax.step == 0) return S >= lo && S < hi;
    const float a0 = __builtin_fmaf(lo, ax.inv, ax.c);
    const float a1 = __builtin_fmaf(hi, ax.inv, ax.c);
    amin = fmaxf(amin, fminf(a0, a1));
    amax = fminf(amax, fmaxf(a0, a1));
    return true;
}

// Cell entered at parameter a along one axis, clamped to [lo, hi - 1]: on a
// plane the ray belongs to the cell it moves into.
__device__ __forceinline__ int entry_cell(float S, float d, float a, int step, int lo, int hi)
{
    const float x = __builtin_fmaf(a, d, S);
    int i = step < 0 ? (int)__builtin_ceilf(x) - 1 : (int)__builtin_floorf(x);
    i = i < lo ? lo : i;
    i = i > hi - 1 ? hi - 1 : i;
    return i;
}

// Cell at parameter a along one axis in the walks' crossing order: the cell
// entered at a (on a plane, the one the ray moves into), moved back by one
// when the FP32 crossing parameter of the plane through which the ray enters
// that cell lies beyond a, then clamped to [lo, hi - 1].  For a ray (nearly)
// parallel to an axis's planes whose FP32 position rounds onto one of them,
// the position and the crossing parameters disagree; the walks step by the
// crossing parameters, so their start cells must follow them too (the
// forward walk and each adjoint brick then split the ray at the same plane).
__device__ __forceinline__ int ordered_cell(const SiddonAxis& ax, float S, float d, float a, int lo, int hi)
{
    const float x = __builtin_fmaf(a, d, S);
    int i = ax.step < 0 ? (int)__builtin_ceilf(x) - 1 : (int)__builtin_floorf(x);
    if (ax.step != 0 && plane_alpha(ax, (float)(i + (ax.step < 0))) > a) i -= ax.step;
    i = i < lo ? lo : i;
    i = i > hi - 1 ? hi - 1 : i;
    return i;
}

// FP64 source and direction of the ray through the centre of pixel (iu, iv).
__device__ __forceinline__ void pixel_ray64(const ViewGeo64& g, int iu, int iv, double S[3], double d[3])
{
    const double fu = (double)iu, fv = (double)iv;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        S[a] = g.S[a];
        d[a] = __builtin_fma(fv, g.DV[a], __builtin_fma(fu, g.DU[a], g.P00[a])) - g.S[a];
    }
}

// Siddon ray X(alpha) = S + alpha d re-anchored at the point of the line
// closest to the volume centre, so that the FP32 plane crossings
// alpha = (q - S) / d are formed from small numbers.  The source -> pixel
// segment is alpha in [a_lo, a_hi].  Forward and adjoint kernels both set up
// rays here.
__device__ __forceinline__ void siddon_ray(const ViewGeo64& g, int iu, int iv, const VolDims& v, float S[3],
                                           float d[3], float& a_lo, float& a_hi)
{
    double Sd[3], dd[3];
    pixel_ray64(g, iu, iv, Sd, dd);
    const double c[3] = {0.5 * v.nx, 0.5 * v.ny, 0.5 * v.nz};
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        num = __builtin_fma(c[a] - Sd[a], dd[a], num);
        den = __builtin_fma(dd[a], dd[a], den);
    }
    const double t0 = num / den;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        S[a] = (float)__builtin_fma(t0, dd[a], Sd[a]);
        d[a] = (float)dd[a];
    }
    a_lo = (float)(-t0);
    a_hi = (float)(1.0 - t0);
}

// Workgroups are handed to the chip's 8 XCDs in turn (workgroup i to XCD
// i mod 8), and each XCD has its own L2.  This renumbering gives every XCD
// one contiguous run of the logical block order, so blocks that read the
// same data run under the same L2.  A bijection on [0, n).
__device__ __forceinline__ int64_t xcd_contiguous(int64_t b, int64_t n)
{
    const int64_t per = n / 8, rem = n % 8;
    const int64_t x = b % 8, i = b / 8;
    return x * per + (x < rem ? x : rem) + i;
}

// --- interpolated ----------------------------------------------------------
// Samples of the ray in voxel-centre coordinates: sample k is at
// base + (k - kc) st, kc the middle sample of k0..k1, the samples inside the
// open box (-1, n) where the trilinear interpolant can be nonzero.  The
// setup (clip, sample range, anchor) is FP64; base and st are rounded once.
struct InterpRay {
    float st[3];   // step per sample, voxel units
    float base[3]; // position of sample kc
    float inv[3];  // rcp(st) where st != 0 (the clip's reciprocals, reusable)
    int kc, k0, k1;
};

// Interpolated-projector ray of pixel (iu, iv): samples k sit at S + k ds d̂
// in voxel-centre coordinates.  [k0, k1] holds every sample whose trilinear
// support (-1, n) per axis can be entered, widened by one sample at each end
// (those extra samples lie at most one step outside the support, where the
// interpolant is 0, so they add nothing); kc = (k0 + k1) / 2 anchors the
// FP32 positions base + (k - kc) st, with base formed in FP64.  The forward
// projector and its transpose both call this function, so they visit the
// same samples at the same FP32 positions.
__device__ __forceinline__ bool interp_ray(const ViewGeo64& g, int iu, int iv, const VolDims& v, float ds,
                                           float inv_ds, InterpRay& r)
{
    // a ray that misses returns with an empty sample range anchored at 0
    r.k0 = 0;
    r.k1 = -1;
    r.kc = 0;
    double S[3], d[3];
    pixel_ray64(g, iu, iv, S, d);
    const double x = d[0] * v.hx, y = d[1] * v.hy, z = d[2] * v.hz;
    const double L2 = __builtin_fma(x, x, __builtin_fma(y, y, z * z));
    // 1 / L: hardware estimate refined by two Newton steps (full FP64 accuracy)
    double rl = __builtin_amdgcn_rsq(L2);
    rl = rl * __builtin_fma(-0.5 * L2, rl * rl, 1.5);
    rl = rl * __builtin_fma(-0.5 * L2, rl * rl, 1.5);
    const double sc = (double)ds * rl;
    const int n[3] = {v.nx, v.ny, v.nz};
    // samples up to the detector pixel (inv_ds = 1 / ds; a bound only:
    // the volume's box below is tighter whenever the volume lies between
    // source and detector)
    float kmin = 0.0f, kmax = (float)(L2 * rl) * inv_ds;
    double Sc[3], st[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Sc[a] = S[a] - 0.5;
        st[a] = d[a] * sc;
        const float stf = (float)st[a], Sf = (float)Sc[a];
        r.inv[a] = 0.0f;
        if (stf != 0.0f) {
            const float inv = __builtin_amdgcn_rcpf(stf);
            r.inv[a] = inv;
            const float ka = (-1.0f - Sf) * inv, kb = ((float)n[a] - Sf) * inv;
            kmin = fmaxf(kmin, fminf(ka, kb));
            kmax = fminf(kmax, fmaxf(ka, kb));
        } else if (!(Sf > -1.0f && Sf < (float)n[a])) {
            return false;
        }
    }
    if (!(kmin <= kmax + 2.0f)) return false;
    r.k0 = (int)__builtin_ceilf(kmin) - 1;
    r.k1 = (int)__builtin_floorf(kmax) + 1;
    if (r.k1 < r.k0) return false;
    r.kc = (r.k0 + r.k1) >> 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.st[a] = (float)st[a];
        r.base[a] = (float)__builtin_fma((double)r.kc, st[a], Sc[a]);
    }
    return true;
}

__device__ __forceinline__ void interp_pos(const InterpRay& r, int k, float p[3])
{
    const float j = (float)(k - r.kc);
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = __builtin_fmaf(j, r.st[a], r.base[a]);
}

#endif  // __HIPCC__

}  // namespace ctmi

// The opaque plan of the C ABI is the library's Plan.
struct ctmi_plan : ctmi::Plan {};
