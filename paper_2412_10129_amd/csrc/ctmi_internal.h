// Internal declarations of libctmi: the device view table, the ray helpers
// that the forward projectors and their transposes share, and the kernel
// launchers.  The forward and adjoint kernels include the same inline
// helpers so that both evaluate every matrix entry with identical FP32
// arithmetic (explicit fmaf, no contraction), which makes the adjoint exact
// up to summation order.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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
    int device;
    ViewGeo* d_views;     // [nviews]
    float* d_filter;      // [fft_len] Ram-Lak response, bit-reversed order, 1/L folded in
    float2* d_twiddle;    // [fft_len / 2] exp(-2 pi i k / L)
    int fft_len;
    int fft_log2;
    VolDims vol;
    DetDims det;
    float ds;             // interpolated-projector step, mm
    float bound_siddon;   // bound on sum_i |a_ij| over the rays of one view, Siddon (mm)
    float bound_interp;   // the same for the interpolated projector (mm)
};

// ------------------------------------------------------------ launchers
hipError_t launch_forward_siddon(const Plan& p, const float* vol, float* proj, int64_t view0, int64_t nviews,
                                 hipStream_t s);
hipError_t launch_forward_interp(const Plan& p, const float* vol, float* proj, int64_t view0, int64_t nviews,
                                 hipStream_t s);
hipError_t launch_backward_siddon(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                                  float beta, hipStream_t s);
hipError_t launch_backward_interp(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                                  float beta, hipStream_t s);
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
hipError_t launch_fov_sq_err(const Plan& p, const float* x, const float* gt, double* out, double* ws,
                             hipStream_t s);

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
        ax.inv = 1.0f / d;
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

// --- interpolated ----------------------------------------------------------
// Samples of the ray in voxel-centre coordinates: pos_k = base + (k - k0) st,
// k0..k1 the samples inside the open box (-1, n) where the trilinear
// interpolant can be nonzero.  `ds` is the step in mm.
struct InterpRay {
    float Sc[3];   // source, voxel-centre coordinates
    float st[3];   // step per sample, voxel units
    float base[3]; // position of sample k0
    int k0, k1;
};

__device__ __forceinline__ bool interp_ray(const ViewGeo& g, int iu, int iv, const VolDims& v, float ds,
                                           InterpRay& r)
{
    float S[3], d[3];
    pixel_ray(g, iu, iv, S, d);
    const float L = world_length(d, v);
    const float scale = ds / L;
    const int n[3] = {v.nx, v.ny, v.nz};
    float kmin = 0.0f, kmax = L / ds;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        r.Sc[a] = S[a] - 0.5f;
        r.st[a] = d[a] * scale;
        if (r.st[a] != 0.0f) {
            const float inv = 1.0f / r.st[a];
            const float ka = (-1.0f - r.Sc[a]) * inv;
            const float kb = ((float)n[a] - r.Sc[a]) * inv;
            kmin = fmaxf(kmin, fminf(ka, kb));
            kmax = fminf(kmax, fmaxf(ka, kb));
        } else if (!(r.Sc[a] > -1.0f && r.Sc[a] < (float)n[a])) {
            return false;
        }
    }
    if (!(kmin < kmax)) return false;
    r.k0 = (int)__builtin_ceilf(kmin);
    r.k1 = (int)__builtin_floorf(kmax);
    const float fk0 = (float)r.k0;
#pragma unroll
    for (int a = 0; a < 3; ++a) r.base[a] = __builtin_fmaf(fk0, r.st[a], r.Sc[a]);
    return r.k1 >= r.k0;
}

__device__ __forceinline__ void interp_pos(const InterpRay& r, int k, float p[3])
{
    const float j = (float)(k - r.k0);
#pragma unroll
    for (int a = 0; a < 3; ++a) p[a] = __builtin_fmaf(j, r.st[a], r.base[a]);
}

#endif  // __HIPCC__

}  // namespace ctmi
