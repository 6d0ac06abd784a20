// Forward projectors A (the linear model A x = b of section 2.1): one thread
// per detector pixel, projection-major ray tiles.
//
// Work decomposition: a workgroup of 256 threads owns a 16x16 pixel tile of
// one view; each wavefront covers an 8x8 sub-tile so the 64 rays of a wave
// travel through neighbouring voxels together.  Blocks are ordered
// (tile row, view, tile column): the workgroups in flight at any moment
// share one detector row band, hence one z-slab of the volume, across many
// views -- that slab stays resident in L2 / Infinity Cache while the views
// stream past it.  Detector writes are one float per ray.
#include "ctmi_internal.h"

namespace ctmi {

namespace {

constexpr int TILE = 16;

struct TileMap {
    int tiles_u, tiles_v;
    int64_t nviews;
};

__device__ __forceinline__ void tile_pixel(const TileMap& m, int64_t b, int& view, int& iu, int& iv)
{
    const int64_t per_row = m.nviews * m.tiles_u;
    const int tv = (int)(b / per_row);
    const int64_t rem = b - (int64_t)tv * per_row;
    view = (int)(rem / m.tiles_u);
    const int tu = (int)(rem - (int64_t)view * m.tiles_u);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    iu = tu * TILE + (w & 1) * 8 + (lane & 7);
    iv = tv * TILE + (w >> 1) * 8 + (lane >> 3);
}

__global__ void __launch_bounds__(256) k_forward_siddon(const float* __restrict__ vol, float* __restrict__ proj,
                                                        const ViewGeo* __restrict__ tab, int view0, TileMap m,
                                                        VolDims v, DetDims det)
{
    int view, iu, iv;
    tile_pixel(m, blockIdx.x, view, iu, iv);
    if (iu >= det.nu || iv >= det.nv) return;
    const ViewGeo& g = tab[view0 + view];

    float S[3], d[3];
    pixel_ray(g, iu, iv, S, d);
    const float L = world_length(d, v);
    const SiddonAxis ax = siddon_axis(S[0], d[0]);
    const SiddonAxis ay = siddon_axis(S[1], d[1]);
    const SiddonAxis az = siddon_axis(S[2], d[2]);
    float amin = 0.0f, amax = 1.0f;
    bool hit = slab_clip(ax, S[0], 0.0f, (float)v.nx, amin, amax);
    hit &= slab_clip(ay, S[1], 0.0f, (float)v.ny, amin, amax);
    hit &= slab_clip(az, S[2], 0.0f, (float)v.nz, amin, amax);
    float acc = 0.0f;
    if (hit && amin < amax) {
        int ix = entry_cell(S[0], d[0], amin, ax.step, 0, v.nx);
        int iy = entry_cell(S[1], d[1], amin, ay.step, 0, v.ny);
        int iz = entry_cell(S[2], d[2], amin, az.step, 0, v.nz);
        // next plane crossed on each axis
        float qx = (float)(ix + (ax.step > 0)), qy = (float)(iy + (ay.step > 0)), qz = (float)(iz + (az.step > 0));
        float anx = plane_alpha(ax, qx), any = plane_alpha(ay, qy), anz = plane_alpha(az, qz);
        const int sx = ax.step, sy = ay.step * v.nx, sz = az.step * v.nx * v.ny;
        int idx = (iz * v.ny + iy) * v.nx + ix;
        float acur = amin;
        const int cap = v.nx + v.ny + v.nz + 3;
        for (int it = 0; it < cap; ++it) {
            const float an = fminf(anx, fminf(any, anz));
            const float ae = fminf(an, amax);
            acc = __builtin_fmaf(fmaxf(ae - acur, 0.0f), vol[idx], acc);
            if (an >= amax) break;
            acur = an;
            if (an == anx) {
                ix += ax.step;
                if ((unsigned)ix >= (unsigned)v.nx) break;
                idx += sx;
                qx += (float)ax.step;
                anx = plane_alpha(ax, qx);
            } else if (an == any) {
                iy += ay.step;
                if ((unsigned)iy >= (unsigned)v.ny) break;
                idx += sy;
                qy += (float)ay.step;
                any = plane_alpha(ay, qy);
            } else {
                iz += az.step;
                if ((unsigned)iz >= (unsigned)v.nz) break;
                idx += sz;
                qz += (float)az.step;
                anz = plane_alpha(az, qz);
            }
        }
    }
    proj[((int64_t)view * det.nv + iv) * det.nu + iu] = acc * L;
}

// Trilinear sample of the volume at voxel-centre coordinates p, zero outside.
__device__ __forceinline__ float trilinear(const float* __restrict__ vol, const VolDims& v, const float p[3])
{
    const float fx = __builtin_floorf(p[0]), fy = __builtin_floorf(p[1]), fz = __builtin_floorf(p[2]);
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    const float ax = p[0] - fx, ay = p[1] - fy, az = p[2] - fz;
    // corner weights are zeroed outside the grid and indices are clamped into
    // it, so every load stays in bounds whatever the sample position
    const float wx0 = (unsigned)ix < (unsigned)v.nx ? 1.0f - ax : 0.0f;
    const float wx1 = (unsigned)(ix + 1) < (unsigned)v.nx ? ax : 0.0f;
    const float wy0 = (unsigned)iy < (unsigned)v.ny ? 1.0f - ay : 0.0f;
    const float wy1 = (unsigned)(iy + 1) < (unsigned)v.ny ? ay : 0.0f;
    const float wz0 = (unsigned)iz < (unsigned)v.nz ? 1.0f - az : 0.0f;
    const float wz1 = (unsigned)(iz + 1) < (unsigned)v.nz ? az : 0.0f;
    const int x0 = min(max(ix, 0), v.nx - 1), x1 = min(max(ix + 1, 0), v.nx - 1);
    const int y0 = min(max(iy, 0), v.ny - 1), y1 = min(max(iy + 1, 0), v.ny - 1);
    const int z0 = min(max(iz, 0), v.nz - 1), z1 = min(max(iz + 1, 0), v.nz - 1);
    const int sxy = v.nx * v.ny;
    const float* r00 = vol + z0 * sxy + y0 * v.nx;
    const float* r01 = vol + z0 * sxy + y1 * v.nx;
    const float* r10 = vol + z1 * sxy + y0 * v.nx;
    const float* r11 = vol + z1 * sxy + y1 * v.nx;
    const float c00 = __builtin_fmaf(wx0, r00[x0], wx1 * r00[x1]);
    const float c01 = __builtin_fmaf(wx0, r01[x0], wx1 * r01[x1]);
    const float c10 = __builtin_fmaf(wx0, r10[x0], wx1 * r10[x1]);
    const float c11 = __builtin_fmaf(wx0, r11[x0], wx1 * r11[x1]);
    const float c0 = __builtin_fmaf(wy0, c00, wy1 * c01);
    const float c1 = __builtin_fmaf(wy0, c10, wy1 * c11);
    return __builtin_fmaf(wz0, c0, wz1 * c1);
}

__global__ void __launch_bounds__(256) k_forward_interp(const float* __restrict__ vol, float* __restrict__ proj,
                                                        const ViewGeo* __restrict__ tab, int view0, TileMap m,
                                                        VolDims v, DetDims det, float ds)
{
    int view, iu, iv;
    tile_pixel(m, blockIdx.x, view, iu, iv);
    if (iu >= det.nu || iv >= det.nv) return;
    const ViewGeo& g = tab[view0 + view];
    InterpRay r;
    float acc = 0.0f;
    if (interp_ray(g, iu, iv, v, ds, r)) {
        for (int k = r.k0; k <= r.k1; ++k) {
            float p[3];
            interp_pos(r, k, p);
            acc += trilinear(vol, v, p);
        }
    }
    proj[((int64_t)view * det.nv + iv) * det.nu + iu] = acc * ds;
}

TileMap tile_map(const Plan& p, int64_t nviews)
{
    TileMap m;
    m.tiles_u = (p.det.nu + TILE - 1) / TILE;
    m.tiles_v = (p.det.nv + TILE - 1) / TILE;
    m.nviews = nviews;
    return m;
}

}  // namespace

hipError_t launch_forward_siddon(const Plan& p, const float* vol, float* proj, int64_t view0, int64_t nviews,
                                 hipStream_t s)
{
    const TileMap m = tile_map(p, nviews);
    const int64_t blocks = (int64_t)m.tiles_u * m.tiles_v * nviews;
    hipLaunchKernelGGL(k_forward_siddon, dim3((unsigned)blocks), dim3(256), 0, s, vol, proj, p.d_views,
                       (int)view0, m, p.vol, p.det);
    return hipGetLastError();
}

hipError_t launch_forward_interp(const Plan& p, const float* vol, float* proj, int64_t view0, int64_t nviews,
                                 hipStream_t s)
{
    const TileMap m = tile_map(p, nviews);
    const int64_t blocks = (int64_t)m.tiles_u * m.tiles_v * nviews;
    hipLaunchKernelGGL(k_forward_interp, dim3((unsigned)blocks), dim3(256), 0, s, vol, proj, p.d_views,
                       (int)view0, m, p.vol, p.det, p.ds);
    return hipGetLastError();
}

}  // namespace ctmi
