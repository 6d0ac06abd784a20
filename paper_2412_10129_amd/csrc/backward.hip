// Matched backprojectors: the exact transposes A^T of the Siddon and the
// interpolated forward projectors (needed by the Krylov methods of section
// 2.2.1, and as the gradient of the autograd operator).
//
// Voxel-driven by bricks: a workgroup owns one BxBxB brick of output voxels
// and accumulates it in LDS over every view of the call; each voxel has one
// writer in global memory and no global atomics are used.  Per view, the
// brick's detector footprint (the bounding box of its projected corners) is
// enumerated; each footprint ray is re-traced inside the brick only, with the
// same FP32 arithmetic as the forward kernel (shared helpers in
// ctmi_internal.h), and its in-brick matrix entries a_ij * y_i are added to
// the LDS accumulators.  Bricks are ordered z-slab-major so the workgroups in
// flight read the same detector row band of every view.
#include "ctmi_internal.h"

namespace ctmi {

namespace {

constexpr int BRICK = 16;

struct BrickMap {
    int nbx, nby, nbz;
};

__device__ __forceinline__ void brick_origin(const BrickMap& m, int b, int& bx, int& by, int& bz)
{
    bx = b % m.nbx;
    const int r = b / m.nbx;
    by = r % m.nby;
    bz = r / m.nby;
}

// Pixel range whose rays may cross the voxel-centre-coordinate box
// [lo, hi] (per axis x, y, z): bounding box of the 8 projected corners,
// widened by one pixel and clamped to the detector.  Returns false if empty.
__device__ __forceinline__ bool footprint(const ViewGeo& g, const float lo[3], const float hi[3],
                                          const DetDims& det, int& u0, int& u1, int& v0, int& v1)
{
    float umin = CTMI_INF, umax = -CTMI_INF, vmin = CTMI_INF, vmax = -CTMI_INF;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const float cx = (q & 1) ? hi[0] : lo[0];
        const float cy = (q & 2) ? hi[1] : lo[1];
        const float cz = (q & 4) ? hi[2] : lo[2];
        const float W = __builtin_fmaf(g.MW[0], cx, __builtin_fmaf(g.MW[1], cy, __builtin_fmaf(g.MW[2], cz, g.MW[3])));
        const float U = __builtin_fmaf(g.MU[0], cx, __builtin_fmaf(g.MU[1], cy, __builtin_fmaf(g.MU[2], cz, g.MU[3])));
        const float V = __builtin_fmaf(g.MV[0], cx, __builtin_fmaf(g.MV[1], cy, __builtin_fmaf(g.MV[2], cz, g.MV[3])));
        const float rw = 1.0f / W;
        umin = fminf(umin, U * rw);
        umax = fmaxf(umax, U * rw);
        vmin = fminf(vmin, V * rw);
        vmax = fmaxf(vmax, V * rw);
    }
    // clamp in float first: the corners may project far outside the detector
    umin = fminf(fmaxf(umin, -2.0f), (float)det.nu + 1.0f);
    vmin = fminf(fmaxf(vmin, -2.0f), (float)det.nv + 1.0f);
    umax = fminf(fmaxf(umax, -2.0f), (float)det.nu + 1.0f);
    vmax = fminf(fmaxf(vmax, -2.0f), (float)det.nv + 1.0f);
    u0 = max((int)__builtin_floorf(umin) - 1, 0);
    v0 = max((int)__builtin_floorf(vmin) - 1, 0);
    u1 = min((int)__builtin_ceilf(umax) + 1, det.nu - 1);
    v1 = min((int)__builtin_ceilf(vmax) + 1, det.nv - 1);
    return u0 <= u1 && v0 <= v1;
}

__device__ __forceinline__ void store_brick(float* __restrict__ vol, const float* acc, const VolDims& v, int x0,
                                            int y0, int z0, float beta)
{
    for (int i = threadIdx.x; i < BRICK * BRICK * BRICK; i += blockDim.x) {
        const int lx = i % BRICK, ly = (i / BRICK) % BRICK, lz = i / (BRICK * BRICK);
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        if (gx >= v.nx || gy >= v.ny || gz >= v.nz) continue;
        float* o = vol + ((int64_t)gz * v.ny + gy) * v.nx + gx;
        *o = beta == 0.0f ? acc[i] : __builtin_fmaf(beta, *o, acc[i]);
    }
}

__global__ void __launch_bounds__(256) k_backward_siddon(const float* __restrict__ proj, float* __restrict__ vol,
                                                         const ViewGeo* __restrict__ tab, int view0, int nviews,
                                                         VolDims v, DetDims det, BrickMap m, float beta)
{
    __shared__ float acc[BRICK * BRICK * BRICK];
    for (int i = threadIdx.x; i < BRICK * BRICK * BRICK; i += blockDim.x) acc[i] = 0.0f;
    int bx, by, bz;
    brick_origin(m, blockIdx.x, bx, by, bz);
    const int x0 = bx * BRICK, y0 = by * BRICK, z0 = bz * BRICK;
    const int x1 = min(x0 + BRICK, v.nx), y1 = min(y0 + BRICK, v.ny), z1 = min(z0 + BRICK, v.nz);
    const float lo[3] = {x0 - 0.5f, y0 - 0.5f, z0 - 0.5f};   // cell box in voxel-centre coordinates
    const float hi[3] = {x1 - 0.5f, y1 - 0.5f, z1 - 0.5f};
    __syncthreads();

    for (int k = 0; k < nviews; ++k) {
        const ViewGeo& g = tab[view0 + k];
        int u0, u1, vv0, vv1;
        if (!footprint(g, lo, hi, det, u0, u1, vv0, vv1)) continue;
        const int w = u1 - u0 + 1;
        const int npx = w * (vv1 - vv0 + 1);
        const float* pk = proj + (int64_t)k * det.nv * det.nu;
        for (int p = threadIdx.x; p < npx; p += blockDim.x) {
            const int r = p / w;
            const int iv = vv0 + r, iu = u0 + (p - r * w);
            float S[3], d[3];
            pixel_ray(g, iu, iv, S, d);
            const SiddonAxis ax = siddon_axis(S[0], d[0]);
            const SiddonAxis ay = siddon_axis(S[1], d[1]);
            const SiddonAxis az = siddon_axis(S[2], d[2]);
            float amin = 0.0f, amax = 1.0f;
            bool hit = slab_clip(ax, S[0], (float)x0, (float)x1, amin, amax);
            hit &= slab_clip(ay, S[1], (float)y0, (float)y1, amin, amax);
            hit &= slab_clip(az, S[2], (float)z0, (float)z1, amin, amax);
            if (!hit || !(amin < amax)) continue;
            const float yl = pk[(int64_t)iv * det.nu + iu] * world_length(d, v);
            int ix = entry_cell(S[0], d[0], amin, ax.step, x0, x1);
            int iy = entry_cell(S[1], d[1], amin, ay.step, y0, y1);
            int iz = entry_cell(S[2], d[2], amin, az.step, z0, z1);
            float qx = (float)(ix + (ax.step > 0)), qy = (float)(iy + (ay.step > 0)), qz = (float)(iz + (az.step > 0));
            float anx = plane_alpha(ax, qx), any = plane_alpha(ay, qy), anz = plane_alpha(az, qz);
            int li = ((iz - z0) * BRICK + (iy - y0)) * BRICK + (ix - x0);
            const int sx = ax.step, sy = ay.step * BRICK, sz = az.step * BRICK * BRICK;
            float acur = amin;
            for (int it = 0; it < 3 * BRICK + 3; ++it) {
                const float an = fminf(anx, fminf(any, anz));
                const float ae = fminf(an, amax);
                atomicAdd(&acc[li], fmaxf(ae - acur, 0.0f) * yl);
                if (an >= amax) break;
                acur = an;
                if (an == anx) {
                    ix += ax.step;
                    if (ix < x0 || ix >= x1) break;
                    li += sx;
                    qx += (float)ax.step;
                    anx = plane_alpha(ax, qx);
                } else if (an == any) {
                    iy += ay.step;
                    if (iy < y0 || iy >= y1) break;
                    li += sy;
                    qy += (float)ay.step;
                    any = plane_alpha(ay, qy);
                } else {
                    iz += az.step;
                    if (iz < z0 || iz >= z1) break;
                    li += sz;
                    qz += (float)az.step;
                    anz = plane_alpha(az, qz);
                }
            }
        }
    }
    __syncthreads();
    store_brick(vol, acc, v, x0, y0, z0, beta);
}

__global__ void __launch_bounds__(256) k_backward_interp(const float* __restrict__ proj, float* __restrict__ vol,
                                                         const ViewGeo* __restrict__ tab, int view0, int nviews,
                                                         VolDims v, DetDims det, BrickMap m, float beta, float ds)
{
    __shared__ float acc[BRICK * BRICK * BRICK];
    for (int i = threadIdx.x; i < BRICK * BRICK * BRICK; i += blockDim.x) acc[i] = 0.0f;
    int bx, by, bz;
    brick_origin(m, blockIdx.x, bx, by, bz);
    const int x0 = bx * BRICK, y0 = by * BRICK, z0 = bz * BRICK;
    const int x1 = min(x0 + BRICK, v.nx), y1 = min(y0 + BRICK, v.ny), z1 = min(z0 + BRICK, v.nz);
    // samples that touch voxels [x0, x1) lie in the open box (x0 - 1, x1) of
    // voxel-centre coordinates
    const float lo[3] = {x0 - 1.0f, y0 - 1.0f, z0 - 1.0f};
    const float hi[3] = {(float)x1, (float)y1, (float)z1};
    const int b0[3] = {x0, y0, z0}, b1[3] = {x1, y1, z1};
    __syncthreads();

    for (int k = 0; k < nviews; ++k) {
        const ViewGeo& g = tab[view0 + k];
        int u0, u1, vv0, vv1;
        if (!footprint(g, lo, hi, det, u0, u1, vv0, vv1)) continue;
        const int w = u1 - u0 + 1;
        const int npx = w * (vv1 - vv0 + 1);
        const float* pk = proj + (int64_t)k * det.nv * det.nu;
        for (int p = threadIdx.x; p < npx; p += blockDim.x) {
            const int r = p / w;
            const int iv = vv0 + r, iu = u0 + (p - r * w);
            InterpRay ray;
            if (!interp_ray(g, iu, iv, v, ds, ray)) continue;
            // sample range inside the brick's box, widened by one sample each
            // side; exact membership is decided per corner below
            float kmin = -CTMI_INF, kmax = CTMI_INF;
            bool inside = true;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                if (ray.st[a] != 0.0f) {
                    const float inv = 1.0f / ray.st[a];
                    const float ka = (lo[a] - ray.Sc[a]) * inv, kb = (hi[a] - ray.Sc[a]) * inv;
                    kmin = fmaxf(kmin, fminf(ka, kb));
                    kmax = fminf(kmax, fmaxf(ka, kb));
                } else {
                    inside &= ray.Sc[a] > lo[a] && ray.Sc[a] < hi[a];
                }
            }
            if (!inside || !(kmin < kmax)) continue;
            const int ks = max(ray.k0, (int)__builtin_ceilf(kmin) - 1);
            const int ke = min(ray.k1, (int)__builtin_floorf(kmax) + 1);
            if (ks > ke) continue;
            const float yds = pk[(int64_t)iv * det.nu + iu] * ds;
            for (int q = ks; q <= ke; ++q) {
                float pos[3];
                interp_pos(ray, q, pos);
                int j0[3];
                float f[3];
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const float fl = __builtin_floorf(pos[a]);
                    j0[a] = (int)fl;
                    f[a] = pos[a] - fl;
                }
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int jx = j0[0] + (c & 1), jy = j0[1] + ((c >> 1) & 1), jz = j0[2] + (c >> 2);
                    if (jx < b0[0] || jx >= b1[0] || jy < b0[1] || jy >= b1[1] || jz < b0[2] || jz >= b1[2]) continue;
                    const float wx = (c & 1) ? f[0] : 1.0f - f[0];
                    const float wy = ((c >> 1) & 1) ? f[1] : 1.0f - f[1];
                    const float wz = (c >> 2) ? f[2] : 1.0f - f[2];
                    atomicAdd(&acc[((jz - z0) * BRICK + (jy - y0)) * BRICK + (jx - x0)], wx * wy * wz * yds);
                }
            }
        }
    }
    __syncthreads();
    store_brick(vol, acc, v, x0, y0, z0, beta);
}

BrickMap brick_map(const Plan& p)
{
    BrickMap m;
    m.nbx = (p.vol.nx + BRICK - 1) / BRICK;
    m.nby = (p.vol.ny + BRICK - 1) / BRICK;
    m.nbz = (p.vol.nz + BRICK - 1) / BRICK;
    return m;
}

}  // namespace

hipError_t launch_backward_siddon(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                                  float beta, hipStream_t s)
{
    const BrickMap m = brick_map(p);
    const unsigned blocks = (unsigned)m.nbx * m.nby * m.nbz;
    hipLaunchKernelGGL(k_backward_siddon, dim3(blocks), dim3(256), 0, s, proj, vol, p.d_views, (int)view0,
                       (int)nviews, p.vol, p.det, m, beta);
    return hipGetLastError();
}

hipError_t launch_backward_interp(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                                  float beta, hipStream_t s)
{
    const BrickMap m = brick_map(p);
    const unsigned blocks = (unsigned)m.nbx * m.nby * m.nbz;
    hipLaunchKernelGGL(k_backward_interp, dim3(blocks), dim3(256), 0, s, proj, vol, p.d_views, (int)view0,
                       (int)nviews, p.vol, p.det, m, beta, p.ds);
    return hipGetLastError();
}

}  // namespace ctmi
