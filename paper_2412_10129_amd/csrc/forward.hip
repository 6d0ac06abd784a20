// Forward projectors A (the linear model A x = b of section 2.1): one thread
// per detector pixel, projection-major ray tiles, LDS-staged volume slabs.
//
// A workgroup of 256 threads owns a 16x16 pixel tile of one view.  The tile's
// rays run mostly along one axis (the dominant axis of the tile's central
// ray); the volume is cut into slabs of SLAB cells across that axis and the
// workgroup visits the slabs in the direction of travel.  For each slab it
// stages in LDS the box of voxels the tile's rays can touch there (bounded by
// the four corner rays of the tile, which enclose the whole ray bundle), then
// every thread advances its own ray through the slab reading the volume from
// LDS.  Global reads are coalesced box loads instead of per-sample gathers
// from scattered cache lines.  A sample whose voxels fall outside the staged
// box (box clipped to the LDS capacity, rounding at the box edge) reads them
// from global memory, so the result never depends on the box estimate.
//
// Blocks are ordered (tile row, groups of 16 views, tile column, view in
// group), and renumbered so that each XCD runs a contiguous run of that
// order: the workgroups in flight on one XCD share one detector row band,
// hence one z-band of the volume, and stage overlapping boxes for nearby
// views under one L2.
//
// The interpolated projector stages its boxes one slab ahead: the next
// slab's first 2048 box elements are loaded into registers while the
// current slab is sampled (7% faster at 512^3 x 720; the register budget is
// held at six waves per SIMD, the LDS limit).  The Siddon walk keeps more
// state per ray and runs slower with the extra registers, so it stages each
// box when it needs it.
#include "ctmi_internal.h"

namespace ctmi {

namespace {

#ifndef CTMI_FWD_TU
#define CTMI_FWD_TU 16
#endif
#ifndef CTMI_FWD_TV
#define CTMI_FWD_TV 16
#endif
#ifndef CTMI_FWD_SLAB
#define CTMI_FWD_SLAB 10
#endif
#ifndef CTMI_FWD_BOXCAP
#define CTMI_FWD_BOXCAP 6144
#endif
// interpolated forward: box elements per thread fetched ahead into
// registers, and the waves per SIMD the register budget is sized for
#ifndef CTMI_FWD_PF
#define CTMI_FWD_PF 8
#endif
#ifndef CTMI_FWD_WAVES
#define CTMI_FWD_WAVES 6
#endif
constexpr int TU = CTMI_FWD_TU, TV = CTMI_FWD_TV;   // ray tile (pixels), TU * TV = 256
constexpr int SLAB = CTMI_FWD_SLAB;                 // slab thickness along the dominant axis
constexpr int BOXCAP = CTMI_FWD_BOXCAP;             // LDS floats for the staged box
static_assert(TU * TV == 256, "one ray per thread");
static_assert(BOXCAP < 65536, "box index must stay below 2^16");

struct TileMap {
    int tiles_u, tiles_v;
    int64_t nviews;
};

// Staged box: voxel index origin and extent per axis (x, y, z); LDS layout
// [z][y][x] with x fastest (coalesced global loads).
struct Box {
    int o[3];
    int e[3];
};

#ifndef CTMI_FWD_XCD
#define CTMI_FWD_XCD 1
#endif
#ifndef CTMI_FWD_ORDER
#define CTMI_FWD_ORDER 1
#endif
#ifndef CTMI_FWD_VG
#define CTMI_FWD_VG 16
#endif

// With CTMI_FWD_XCD each XCD runs a contiguous run of the tile order, so
// tiles that stage overlapping volume boxes (neighbouring tiles of nearby
// views) share an L2 (A 640 -> 582 ms, Siddon 690 -> 592 ms at 512^3 x 720).
__device__ __forceinline__ int64_t xcd_order(int64_t b, int64_t nblocks)
{
    return CTMI_FWD_XCD ? xcd_contiguous(b, nblocks) : b;
}

__device__ __forceinline__ void tile_of_block(const TileMap& m, int64_t b, int& view, int& tu0, int& tv0)
{
    b = xcd_order(b, (int64_t)m.tiles_u * m.tiles_v * m.nviews);
    int tu, tv;
    if (CTMI_FWD_ORDER == 0) {
        // (tile row, view, tile column)
        const int64_t per_row = m.nviews * m.tiles_u;
        tv = (int)(b / per_row);
        const int64_t rem = b - (int64_t)tv * per_row;
        view = (int)(rem / m.tiles_u);
        tu = (int)(rem - (int64_t)view * m.tiles_u);
    } else {
        // (tile row, groups of VG views, tile column, view in group)
        const int64_t per_row = m.nviews * m.tiles_u;
        tv = (int)(b / per_row);
        int64_t rem = b - (int64_t)tv * per_row;
        const int64_t gsz = (int64_t)CTMI_FWD_VG * m.tiles_u;
        const int64_t g = rem / gsz;
        rem -= g * gsz;
        const int64_t nvg = min((int64_t)CTMI_FWD_VG, m.nviews - g * CTMI_FWD_VG);   // views in this group
        tu = (int)(rem / nvg);
        view = (int)(g * CTMI_FWD_VG + (rem - (int64_t)tu * nvg));
    }
    tu0 = tu * TU;
    tv0 = tv * TV;
}

// Dominant axis and travel direction of the tile's central ray (uniform).
__device__ __forceinline__ void tile_axis(const ViewGeo& g, const DetDims& det, int tu0, int tv0, int& a, int& dir)
{
    const float uc = (float)tu0 + 0.5f * (float)(min(TU, det.nu - tu0) - 1);
    const float vc = (float)tv0 + 0.5f * (float)(min(TV, det.nv - tv0) - 1);
    float dc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) dc[i] = g.P00[i] + uc * g.DU[i] + vc * g.DV[i] - g.S[i];
    const float ax = fabsf(dc[0]), ay = fabsf(dc[1]), az = fabsf(dc[2]);
    a = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
    dir = dc[a] >= 0.0f ? 1 : -1;
}

// Bounds along the two non-dominant axes of the tile's ray bundle between
// planes pa0 and pa1 of axis a, in coordinates shifted by `shift` (0 for
// voxel-cell coordinates, 0.5 for voxel-centre coordinates).
__device__ __forceinline__ void bundle_bounds(const ViewGeo& g, const DetDims& det, int tu0, int tv0, int a,
                                              float pa0, float pa1, float shift, float lo[3], float hi[3])
{
    const int iu1 = min(tu0 + TU, det.nu) - 1, iv1 = min(tv0 + TV, det.nv) - 1;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        lo[i] = CTMI_INF;
        hi[i] = -CTMI_INF;
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        float S[3], d[3];
        pixel_ray(g, (c & 1) ? iu1 : tu0, (c & 2) ? iv1 : tv0, S, d);
#pragma unroll
        for (int i = 0; i < 3; ++i) S[i] -= shift;
        const float inv = 1.0f / d[a];
#pragma unroll
        for (int pl = 0; pl < 2; ++pl) {
            const float t = ((pl ? pa1 : pa0) - S[a]) * inv;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float x = __builtin_fmaf(t, d[i], S[i]);
                lo[i] = fminf(lo[i], x);
                hi[i] = fmaxf(hi[i], x);
            }
        }
    }
}

// Box covering index range [lo_i, hi_i] per axis, clipped to [clo_i, chi_i]
// and to the LDS capacity (the non-dominant axes shrink first).  Returns
// false if empty.
__device__ __forceinline__ bool make_box(const int lo[3], const int hi[3], const int clo[3], const int chi[3], int a,
                                         Box& b)
{
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        const int l = max(lo[i], clo[i]), h = min(hi[i], chi[i]);
        if (h < l) return false;
        b.o[i] = l;
        b.e[i] = h - l + 1;
    }
    // capacity: shrink the larger non-dominant extent until the box fits
    // (every index below is a compile-time constant, so the box stays in
    // registers)
    for (int it = 0; it < 4 && b.e[0] * b.e[1] * b.e[2] > BOXCAP; ++it) {
        const int e1 = a == 0 ? b.e[1] : b.e[0];      // first non-dominant extent
        const int e2 = a == 2 ? b.e[1] : b.e[2];      // second non-dominant extent
        const bool first = e1 >= e2;
        const int keep = first ? e2 : e1;             // the other non-dominant extent
        const int ea = a == 0 ? b.e[0] : (a == 1 ? b.e[1] : b.e[2]);
        const int ne = max(1, BOXCAP / (keep * ea));
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const bool is1 = i == (a == 0 ? 1 : 0), is2 = i == (a == 2 ? 1 : 2);
            if ((first && is1) || (!first && is2)) b.e[i] = ne;
        }
    }
    return b.e[0] * b.e[1] * b.e[2] <= BOXCAP;
}

// Flat loop over the box with x fastest (coalesced global reads).  The
// index is split into (x, y, z) with float reciprocals: floor((i + 1/2) r),
// r = fl(1/e), equals i / e for every i < 2^22, because (i + 1/2)/e is at
// least 1/(2e) away from an integer while the FP32 error is below
// (i + 1/2) 2^-23 / e.
__device__ __forceinline__ void load_box(float* box, const float* __restrict__ vol, const VolDims& v, const Box& b)
{
    const int n = b.e[0] * b.e[1] * b.e[2];
    const float r0 = 1.0f / (float)b.e[0], r1 = 1.0f / (float)b.e[1];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        const int r = (int)__builtin_floorf(((float)i + 0.5f) * r0);
        const int lx = i - (int)__umul24(r, b.e[0]);
        const int lz = (int)__builtin_floorf(((float)r + 0.5f) * r1);
        const int ly = r - (int)__umul24(lz, b.e[1]);
        const int gx = b.o[0] + lx, gy = b.o[1] + ly, gz = b.o[2] + lz;
        float val = 0.0f;
        // the volume has fewer than 2^31 voxels (checked at plan creation), so
        // the linear index fits 32 bits
        if ((unsigned)gx < (unsigned)v.nx && (unsigned)gy < (unsigned)v.ny && (unsigned)gz < (unsigned)v.nz)
            val = vol[(__umul24((unsigned)gz, (unsigned)v.ny) + (unsigned)gy) * (unsigned)v.nx + (unsigned)gx];
        box[i] = val;
    }
}

// Software-pipelined staging: the first PF * 256 elements of the next slab's
// box are loaded into registers (element i = threadIdx.x + 256 m in
// r[m]) while the current slab is sampled, then written to LDS; any
// elements beyond that are read directly when the box is written.  Same
// index split as load_box.
template <int PF>
__device__ __forceinline__ void fetch_box(float (&r)[PF], const float* __restrict__ vol, const VolDims& v,
                                          const Box& b, bool on)
{
    const int n = on ? b.e[0] * b.e[1] * b.e[2] : 0;
    const float r0 = 1.0f / (float)b.e[0], r1 = 1.0f / (float)b.e[1];
#pragma unroll
    for (int m = 0; m < PF; ++m) {
        const int i = (int)threadIdx.x + 256 * m;
        float val = 0.0f;
        if (i < n) {
            const int q = (int)__builtin_floorf(((float)i + 0.5f) * r0);
            const int lx = i - (int)__umul24(q, b.e[0]);
            const int lz = (int)__builtin_floorf(((float)q + 0.5f) * r1);
            const int ly = q - (int)__umul24(lz, b.e[1]);
            const int gx = b.o[0] + lx, gy = b.o[1] + ly, gz = b.o[2] + lz;
            if ((unsigned)gx < (unsigned)v.nx && (unsigned)gy < (unsigned)v.ny && (unsigned)gz < (unsigned)v.nz)
                val = vol[(__umul24((unsigned)gz, (unsigned)v.ny) + (unsigned)gy) * (unsigned)v.nx + (unsigned)gx];
        }
        r[m] = val;
    }
}

template <int PF>
__device__ __forceinline__ void put_box(float* box, const float (&r)[PF], const float* __restrict__ vol,
                                        const VolDims& v, const Box& b, bool on)
{
    const int n = on ? b.e[0] * b.e[1] * b.e[2] : 0;
#pragma unroll
    for (int m = 0; m < PF; ++m) {
        const int i = (int)threadIdx.x + 256 * m;
        if (i < n) box[i] = r[m];
    }
    if (n > 256 * PF) {
        const float r0 = 1.0f / (float)b.e[0], r1 = 1.0f / (float)b.e[1];
        for (int i = (int)threadIdx.x + 256 * PF; i < n; i += 256) {
            const int q = (int)__builtin_floorf(((float)i + 0.5f) * r0);
            const int lx = i - (int)__umul24(q, b.e[0]);
            const int lz = (int)__builtin_floorf(((float)q + 0.5f) * r1);
            const int ly = q - (int)__umul24(lz, b.e[1]);
            const int gx = b.o[0] + lx, gy = b.o[1] + ly, gz = b.o[2] + lz;
            float val = 0.0f;
            if ((unsigned)gx < (unsigned)v.nx && (unsigned)gy < (unsigned)v.ny && (unsigned)gz < (unsigned)v.nz)
                val = vol[(__umul24((unsigned)gz, (unsigned)v.ny) + (unsigned)gy) * (unsigned)v.nx + (unsigned)gx];
            box[i] = val;
        }
    }
}

// ------------------------------------------------------------------ Siddon
struct SiddonWalk {
    int ix, iy, iz, idx;
    float qx, qy, qz, anx, any, anz, acur, amax, acc;
    int left;  // iteration budget
    bool alive;
};

__global__ void __launch_bounds__(256) k_forward_siddon(const float* __restrict__ vol, float* __restrict__ proj,
                                                        const ViewGeo* __restrict__ tab,
                                                        const ViewGeo64* __restrict__ tab64, int view0, TileMap m,
                                                        VolDims v, DetDims det)
{
    __shared__ float box[BOXCAP];
    int view, tu0, tv0;
    tile_of_block(m, blockIdx.x, view, tu0, tv0);
    const int iu = tu0 + (int)(threadIdx.x % TU), iv = tv0 + (int)(threadIdx.x / TU);
    const bool active = iu < det.nu && iv < det.nv;
    const ViewGeo& g = tab[view0 + view];

    float S[3], d[3], a_lo, a_hi;
    siddon_ray(tab64[view0 + view], active ? iu : 0, active ? iv : 0, v, S, d, a_lo, a_hi);
    const float L = world_length(d, v);
    const SiddonAxis ax = siddon_axis(S[0], d[0]);
    const SiddonAxis ay = siddon_axis(S[1], d[1]);
    const SiddonAxis az = siddon_axis(S[2], d[2]);
    SiddonWalk w;
    w.acc = 0.0f;
    w.amax = a_hi;
    float amin = a_lo;
    bool hit = slab_clip(ax, S[0], 0.0f, (float)v.nx, amin, w.amax);
    hit &= slab_clip(ay, S[1], 0.0f, (float)v.ny, amin, w.amax);
    hit &= slab_clip(az, S[2], 0.0f, (float)v.nz, amin, w.amax);
    w.alive = active && hit && amin < w.amax;
    w.ix = ordered_cell(ax, S[0], d[0], amin, 0, v.nx);
    w.iy = ordered_cell(ay, S[1], d[1], amin, 0, v.ny);
    w.iz = ordered_cell(az, S[2], d[2], amin, 0, v.nz);
    w.qx = (float)(w.ix + (ax.step > 0));
    w.qy = (float)(w.iy + (ay.step > 0));
    w.qz = (float)(w.iz + (az.step > 0));
    w.anx = plane_alpha(ax, w.qx);
    w.any = plane_alpha(ay, w.qy);
    w.anz = plane_alpha(az, w.qz);
    w.idx = (w.iz * v.ny + w.iy) * v.nx + w.ix;
    w.acur = amin;
    w.left = v.nx + v.ny + v.nz + 3;
    const int sx = ax.step, sy = ay.step * v.nx, sz = az.step * v.nx * v.ny;

    int a, dir;
    tile_axis(g, det, tu0, tv0, a, dir);
    const int na = a == 0 ? v.nx : (a == 1 ? v.ny : v.nz);
    const int nslab = (na + SLAB - 1) / SLAB;
    const int clo[3] = {0, 0, 0}, chi[3] = {v.nx - 1, v.ny - 1, v.nz - 1};

    for (int si = 0; si < nslab; ++si) {
        const int s = dir > 0 ? si : nslab - 1 - si;
        const int c0 = s * SLAB, c1 = min(c0 + SLAB, na);   // cells [c0, c1) along a
        float blo[3], bhi[3];
        bundle_bounds(g, det, tu0, tv0, a, (float)c0, (float)c1, 0.0f, blo, bhi);
        int lo[3], hi[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lo[i] = (int)__builtin_floorf(fmaxf(blo[i], -4.0f)) - 1;
            hi[i] = (int)__builtin_floorf(fminf(bhi[i], 1.0e7f)) + 1;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lo[i] = i == a ? c0 : lo[i];
            hi[i] = i == a ? c1 - 1 : hi[i];
        }
        Box b;
        if (!make_box(lo, hi, clo, chi, a, b)) continue;
        __syncthreads();
        load_box(box, vol, v, b);
        __syncthreads();
        if (w.alive) {
            // walk the slab on box coordinates: the LDS offset follows the
            // cell, each step advances the crossing axis by selects (no
            // divergent branches), and a cell outside the box (a box clipped
            // to the LDS capacity) is read from global memory instead
            int lx = w.ix - b.o[0], ly = w.iy - b.o[1], lz = w.iz - b.o[2];
            int loff = (lz * b.e[1] + ly) * b.e[0] + lx;
            const int ox = ax.step, oy = ay.step * b.e[0], oz = az.step * b.e[0] * b.e[1];
            const float fx = (float)ax.step, fy = (float)ay.step, fz = (float)az.step;
            for (;;) {
                // the ray has left this slab once its dominant coordinate leaves the box
                const int ld = a == 0 ? lx : (a == 1 ? ly : lz);
                const int ed = a == 0 ? b.e[0] : (a == 1 ? b.e[1] : b.e[2]);
                if ((unsigned)ld >= (unsigned)ed) break;
                const bool in = (unsigned)lx < (unsigned)b.e[0] && (unsigned)ly < (unsigned)b.e[1] &&
                                (unsigned)lz < (unsigned)b.e[2];
                float val = box[in ? loff : 0];
                // keep the LDS read a plain ds_read: the global fallback below
                // must not be merged with it into one generic (flat) load
                asm volatile("" : "+v"(val));
                if (!in) val = vol[w.idx];
                const float an = fminf(w.anx, fminf(w.any, w.anz));
                const float ae = fminf(an, w.amax);
                w.acc = __builtin_fmaf(fmaxf(ae - w.acur, 0.0f), val, w.acc);
                if (an >= w.amax || --w.left <= 0) {
                    w.alive = false;
                    break;
                }
                w.acur = an;
                const bool mx = an == w.anx, my = !mx && an == w.any, mz = !mx && !my;
                lx += mx ? ax.step : 0;
                ly += my ? ay.step : 0;
                lz += mz ? az.step : 0;
                loff += mx ? ox : (my ? oy : oz);
                w.idx += mx ? sx : (my ? sy : sz);
                w.qx += mx ? fx : 0.0f;
                w.qy += my ? fy : 0.0f;
                w.qz += mz ? fz : 0.0f;
                w.anx = mx ? plane_alpha(ax, w.qx) : w.anx;
                w.any = my ? plane_alpha(ay, w.qy) : w.any;
                w.anz = mz ? plane_alpha(az, w.qz) : w.anz;
            }
            w.ix = lx + b.o[0];
            w.iy = ly + b.o[1];
            w.iz = lz + b.o[2];
            // a step out of the volume ends the ray (it crosses the volume's
            // face at amax, so this only guards rounding)
            if ((unsigned)w.ix >= (unsigned)v.nx || (unsigned)w.iy >= (unsigned)v.ny ||
                (unsigned)w.iz >= (unsigned)v.nz)
                w.alive = false;
        }
    }
    // anything left (never expected) finishes from global memory
    while (w.alive) {
        const float an = fminf(w.anx, fminf(w.any, w.anz));
        const float ae = fminf(an, w.amax);
        w.acc = __builtin_fmaf(fmaxf(ae - w.acur, 0.0f), vol[w.idx], w.acc);
        if (an >= w.amax || --w.left <= 0) break;
        w.acur = an;
        if (an == w.anx) {
            w.ix += ax.step;
            if ((unsigned)w.ix >= (unsigned)v.nx) break;
            w.idx += sx;
            w.qx += (float)ax.step;
            w.anx = plane_alpha(ax, w.qx);
        } else if (an == w.any) {
            w.iy += ay.step;
            if ((unsigned)w.iy >= (unsigned)v.ny) break;
            w.idx += sy;
            w.qy += (float)ay.step;
            w.any = plane_alpha(ay, w.qy);
        } else {
            w.iz += az.step;
            if ((unsigned)w.iz >= (unsigned)v.nz) break;
            w.idx += sz;
            w.qz += (float)az.step;
            w.anz = plane_alpha(az, w.qz);
        }
    }
    if (active) proj[((int64_t)view * det.nv + iv) * det.nu + iu] = w.acc * L;
}

// ------------------------------------------------------------ interpolated
__device__ __forceinline__ float lerp1(float a, float r0, float r1) { return __builtin_fmaf(a, r1 - r0, r0); }

// Trilinear sample of the volume at voxel-centre coordinates p, zero outside
// the grid (out-of-grid corners read as 0, indices clamped so every load is
// in bounds).  Same lerp sequence as the LDS path, so both give the same bits.
__device__ __forceinline__ float trilinear_global(const float* __restrict__ vol, const VolDims& v, const float p[3])
{
    const float fx = __builtin_floorf(p[0]), fy = __builtin_floorf(p[1]), fz = __builtin_floorf(p[2]);
    const int ix = (int)fx, iy = (int)fy, iz = (int)fz;
    const float ax = p[0] - fx, ay = p[1] - fy, az = p[2] - fz;
    float r[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int jx = ix + (c & 1), jy = iy + ((c >> 1) & 1), jz = iz + (c >> 2);
        const bool in = (unsigned)jx < (unsigned)v.nx && (unsigned)jy < (unsigned)v.ny && (unsigned)jz < (unsigned)v.nz;
        const int cx = min(max(jx, 0), v.nx - 1), cy = min(max(jy, 0), v.ny - 1), cz = min(max(jz, 0), v.nz - 1);
        const float val = vol[((int64_t)cz * v.ny + cy) * v.nx + cx];
        r[c] = in ? val : 0.0f;
    }
    const float c00 = lerp1(ax, r[0], r[1]), c01 = lerp1(ax, r[2], r[3]);
    const float c10 = lerp1(ax, r[4], r[5]), c11 = lerp1(ax, r[6], r[7]);
    return lerp1(az, lerp1(ay, c00, c01), lerp1(ay, c10, c11));
}

// Per-tile ray-bundle description in LDS: for each corner ray c and axis i,
// the coordinate on plane P of the dominant axis is K[c][i] + P * G[c][i].
struct Bundle {
    float K[4][3], G[4][3];
};

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CTMI_FWD_WAVES, 8))) k_forward_interp(const float* __restrict__ vol, float* __restrict__ proj,
                                                        const ViewGeo* __restrict__ tab,
                                                        const ViewGeo64* __restrict__ tab64, int view0, TileMap m,
                                                        VolDims v, DetDims det, float ds)
{
    __shared__ float box[BOXCAP];
    __shared__ Bundle bun;
    int view, tu0, tv0;
    tile_of_block(m, blockIdx.x, view, tu0, tv0);
    const int iu = tu0 + (int)(threadIdx.x % TU), iv = tv0 + (int)(threadIdx.x / TU);
    const bool active = iu < det.nu && iv < det.nv;
    const ViewGeo& g = tab[view0 + view];
    int a, dir;
    tile_axis(g, det, tu0, tv0, a, dir);
    if (threadIdx.x < 4) {
        // corner rays of the tile, voxel-centre coordinates
        const int c = threadIdx.x;
        const int cu = (c & 1) ? min(tu0 + TU, det.nu) - 1 : tu0, cv = (c & 2) ? min(tv0 + TV, det.nv) - 1 : tv0;
        float S[3], d[3];
        pixel_ray(g, cu, cv, S, d);
        const float inv = 1.0f / d[a];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            const float Gi = d[i] * inv;
            bun.G[c][i] = Gi;
            bun.K[c][i] = (S[i] - 0.5f) - (S[a] - 0.5f) * Gi;
        }
    }

    InterpRay r;
    const bool has = interp_ray(tab64[view0 + view], active ? iu : 0, active ? iv : 0, v, ds, 1.0f / ds, r) && active;
    int k = has ? r.k0 : 0;
    const int k1 = has ? r.k1 : -1;
    // sample k sits at base + (k - kc) st; along the dominant axis the slab
    // boundary plane P is reached at (k - kc) = (P - base_a) / st_a
    const float sa = a == 0 ? r.st[0] : (a == 1 ? r.st[1] : r.st[2]);
    const float ba = a == 0 ? r.base[0] : (a == 1 ? r.base[1] : r.base[2]);
    // the slab bookkeeping needs the ray to advance along the tile's direction
    // (always true for tile-sized bundles); any other ray takes the checked
    // path in the first slab
    const bool mono = dir > 0 ? sa > 1e-6f : sa < -1e-6f;
    const float inv_sa = mono ? 1.0f / sa : 0.0f;
    float acc = 0.0f;
    __syncthreads();

    const int na = a == 0 ? v.nx : (a == 1 ? v.ny : v.nz);
    // a sample's lower corner A = floor(pos_a) lies in [-2, n] (the sample
    // range reaches one step beyond the interpolant's support, and FP32
    // positions may round across its edge); slab s takes the samples before
    // the plane s SLAB + SLAB - 1 (direction +) or from the plane s SLAB - 1
    // on (direction -), and stages planes [s SLAB - 2, s SLAB + SLAB] so a
    // sample assigned one step early or late by rounding still finds its
    // corners in the box.  Boxes may reach one plane of zeros beyond each
    // halo plane, so every corner of such a sample is staged.
    const int nslab = (na + SLAB) / SLAB;
    const int clo[3] = {-2, -2, -2}, chi[3] = {v.nx + 1, v.ny + 1, v.nz + 1};

    // slab si's plane range [A0, A1], its staged box and whether the box
    // holds the whole bundle range (uniform over the block)
    auto slab_box = [&](int si, int& A0, int& A1, Box& b, bool& fits, bool& clipped) {
        const int s = dir > 0 ? si : nslab - 1 - si;
        A0 = s * SLAB - 1;
        A1 = A0 + SLAB;
        // bundle bounds over the staged plane range [A0 - 1, A1 + 1]
        float blo[3] = {CTMI_INF, CTMI_INF, CTMI_INF}, bhi[3] = {-CTMI_INF, -CTMI_INF, -CTMI_INF};
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const float x0 = __builtin_fmaf((float)(A0 - 1), bun.G[c][i], bun.K[c][i]);
                const float x1 = __builtin_fmaf((float)(A1 + 1), bun.G[c][i], bun.K[c][i]);
                blo[i] = fminf(blo[i], fminf(x0, x1));
                bhi[i] = fmaxf(bhi[i], fmaxf(x0, x1));
            }
        int lo[3], hi[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lo[i] = (int)__builtin_floorf(fmaxf(blo[i], -4.0f)) - 1;
            hi[i] = (int)__builtin_floorf(fminf(bhi[i], 1.0e7f)) + 2;
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lo[i] = i == a ? A0 - 1 : lo[i];
            hi[i] = i == a ? A1 + 1 : hi[i];
        }
        fits = make_box(lo, hi, clo, chi, a, b);
        clipped = false;
        if (fits) {
#pragma unroll
            for (int i = 0; i < 3; ++i) clipped |= b.o[i] > max(lo[i], clo[i]) || b.o[i] + b.e[i] - 1 < min(hi[i], chi[i]);
        }
    };
    // the next slab's box is fetched into registers while this one is sampled
    constexpr int PF = CTMI_FWD_PF;
    float pf[PF];
    int nA0, nA1;
    Box nb;
    bool nfits, nclipped;
    slab_box(0, nA0, nA1, nb, nfits, nclipped);
    fetch_box<PF>(pf, vol, v, nb, nfits);

    for (int si = 0; si < nslab; ++si) {
        const int A0 = nA0, A1 = nA1;
        const Box b = nb;
        const bool fits = nfits, clipped = nclipped;
        // this thread's last sample in the slab
        int kl;
        {
            const float P = dir > 0 ? (float)A1 : (float)A0;
            const float t = (P - ba) * inv_sa;
            kl = r.kc + (dir > 0 ? (int)__builtin_ceilf(t) - 1 : (int)__builtin_floorf(t));
            kl = (si == nslab - 1 || !mono) ? k1 : min(kl, k1);
        }
        __syncthreads();
        put_box<PF>(box, pf, vol, v, b, fits);
        __syncthreads();
        if (si + 1 < nslab) {
            slab_box(si + 1, nA0, nA1, nb, nfits, nclipped);
            fetch_box<PF>(pf, vol, v, nb, nfits);
        }
        if (fits && !clipped && mono) {
            // fast path: every sample of the slab has its 2x2x2 corners in the
            // box; the byte offset is formed in FP32 from box-relative
            // coordinates, every intermediate an integer below 2^24
            const float SY = (float)(4 * b.e[0]), SZ = (float)(4 * b.e[0] * b.e[1]);
            const float ox = (float)b.o[0], oyf = (float)b.o[1], ozf = (float)b.o[2];
            const int oy = 4 * b.e[0], oz = 4 * b.e[0] * b.e[1];
            const char* base = reinterpret_cast<const char*>(box);
            for (; k <= kl; ++k) {
                float p[3];
                interp_pos(r, k, p);
                const float fx = __builtin_floorf(p[0]), fy = __builtin_floorf(p[1]), fz = __builtin_floorf(p[2]);
                const int off = (int)__builtin_fmaf(fz - ozf, SZ, __builtin_fmaf(fy - oyf, SY, (fx - ox) * 4.0f));
                const float* r0 = reinterpret_cast<const float*>(base + off);
                const float* r1 = reinterpret_cast<const float*>(base + off + oy);
                const float* r2 = reinterpret_cast<const float*>(base + off + oz);
                const float* r3 = reinterpret_cast<const float*>(base + off + oz + oy);
                const float ax = p[0] - fx, ay = p[1] - fy, az = p[2] - fz;
                const float c00 = lerp1(ax, r0[0], r0[1]), c01 = lerp1(ax, r1[0], r1[1]);
                const float c10 = lerp1(ax, r2[0], r2[1]), c11 = lerp1(ax, r3[0], r3[1]);
                acc += lerp1(az, lerp1(ay, c00, c01), lerp1(ay, c10, c11));
            }
        } else {
            for (; k <= kl; ++k) {
                float p[3];
                interp_pos(r, k, p);
                const float fx = __builtin_floorf(p[0]), fy = __builtin_floorf(p[1]), fz = __builtin_floorf(p[2]);
                const int lx = (int)fx - b.o[0], ly = (int)fy - b.o[1], lz = (int)fz - b.o[2];
                if (fits && (unsigned)lx < (unsigned)(b.e[0] - 1) && (unsigned)ly < (unsigned)(b.e[1] - 1) &&
                    (unsigned)lz < (unsigned)(b.e[2] - 1)) {
                    const float* q = box + (lz * b.e[1] + ly) * b.e[0] + lx;
                    const int sy = b.e[0], sz = b.e[0] * b.e[1];
                    const float ax = p[0] - fx, ay = p[1] - fy, az = p[2] - fz;
                    const float c00 = lerp1(ax, q[0], q[1]), c01 = lerp1(ax, q[sy], q[sy + 1]);
                    const float c10 = lerp1(ax, q[sz], q[sz + 1]), c11 = lerp1(ax, q[sz + sy], q[sz + sy + 1]);
                    acc += lerp1(az, lerp1(ay, c00, c01), lerp1(ay, c10, c11));
                } else {
                    acc += trilinear_global(vol, v, p);
                }
            }
        }
    }
    for (; k <= k1; ++k) {   // anything left (never expected) reads global memory
        float p[3];
        interp_pos(r, k, p);
        acc += trilinear_global(vol, v, p);
    }
    if (active) proj[((int64_t)view * det.nv + iv) * det.nu + iu] = acc * ds;
}

TileMap tile_map(const Plan& p, int64_t nviews)
{
    TileMap m;
    m.tiles_u = (p.det.nu + TU - 1) / TU;
    m.tiles_v = (p.det.nv + TV - 1) / TV;
    m.nviews = nviews;
    return m;
}

}  // namespace

hipError_t launch_forward_siddon(const Plan& p, const float* vol, float* proj, int64_t view0, int64_t nviews,
                                 hipStream_t s)
{
    const TileMap m = tile_map(p, nviews);
    const int64_t blocks = (int64_t)m.tiles_u * m.tiles_v * nviews;
    hipLaunchKernelGGL(k_forward_siddon, dim3((unsigned)blocks), dim3(256), 0, s, vol, proj, p.d_views, p.d_views64,
                       (int)view0, m, p.vol, p.det);
    return hipGetLastError();
}

hipError_t launch_forward_interp(const Plan& p, const float* vol, float* proj, int64_t view0, int64_t nviews,
                                 hipStream_t s)
{
    const TileMap m = tile_map(p, nviews);
    const int64_t blocks = (int64_t)m.tiles_u * m.tiles_v * nviews;
    hipLaunchKernelGGL(k_forward_interp, dim3((unsigned)blocks), dim3(256), 0, s, vol, proj, p.d_views, p.d_views64,
                       (int)view0, m, p.vol, p.det, p.ds);
    return hipGetLastError();
}

}  // namespace ctmi
