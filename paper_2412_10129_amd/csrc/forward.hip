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
// Siddon forward: waves per SIMD the register budget is sized for
#ifndef CTMI_FWD_SID_WAVES
#define CTMI_FWD_SID_WAVES 6
#endif
constexpr int TU = CTMI_FWD_TU, TV = CTMI_FWD_TV;   // ray tile (pixels), TU * TV = 256
#ifndef CTMI_FWD_SID_SLAB
#define CTMI_FWD_SID_SLAB 12
#endif
constexpr int SLAB = CTMI_FWD_SLAB;                 // slab thickness along the dominant axis (interpolated)
constexpr int SID_SLAB = CTMI_FWD_SID_SLAB;         // the same for the Siddon layer walk
constexpr int BOXCAP = CTMI_FWD_BOXCAP;             // LDS floats for the staged box
constexpr int SLABTAB = 64;                         // slab boxes formed up front per block
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

// Box staging by rows.  A row is the box's x extent W = e[0] at one (y, z);
// thread t takes column t mod W of rows t div W + m RG (pass m), RG =
// floor(256 / W) whole rows per pass, so consecutive threads load
// consecutive x (coalesced global reads, consecutive LDS words) and a
// thread's column and its x bounds check stay fixed.  From one pass to the
// next a thread's row advances by RG = RGz e[1] + RGy, so its (y, z) and its
// global index advance by constants, with one carry from y into z.  Initial
// quotients use float reciprocals: floor((i + 1/2) r), r = fl(1/e), equals
// i div e for every i < 2^22, because (i + 1/2)/e is at least 1/(2e) away
// from an integer while the FP32 error is below (i + 1/2) 2^-23 / e.  The
// global index is kept modulo 2^32 (a cell inside the volume has an index
// below 2^31, checked at plan creation).  A box wider than 256 along x (not
// produced by tile-sized bundles) is staged element by element.
struct Stage {
    int ly, lz;        // this thread's current row as box (y, z); lz >= e[2] once past the last row
    unsigned gi;       // global index of the current element (mod 2^32)
    int li;            // its LDS index
    int rgy, rgz;      // pass advance
    unsigned d1, d2;   // global index advance, and the extra on a carry into z
    int lstep;         // LDS index advance
    bool xok;          // this thread holds a column, inside the volume along x
};

__device__ __forceinline__ Stage stage_of(const Box& b, const VolDims& v)
{
    Stage s;
    const float r0 = 1.0f / (float)b.e[0], r1 = 1.0f / (float)b.e[1];
    const int rg = (int)__builtin_floorf(256.5f * r0);
    const int t = (int)threadIdx.x;
    const int tr = (int)__builtin_floorf(((float)t + 0.5f) * r0);
    const int tx = t - tr * b.e[0];
    s.lz = (int)__builtin_floorf(((float)tr + 0.5f) * r1);
    s.ly = tr - s.lz * b.e[1];
    if (tr >= rg) s.lz = b.e[2];   // no column for this thread
    s.rgz = (int)__builtin_floorf(((float)rg + 0.5f) * r1);
    s.rgy = rg - s.rgz * b.e[1];
    const unsigned nx = (unsigned)v.nx, nxy = (unsigned)v.nx * (unsigned)v.ny;
    const int gx = b.o[0] + tx;
    s.xok = (unsigned)gx < nx;
    s.gi = (unsigned)(b.o[2] + s.lz) * nxy + (unsigned)(b.o[1] + s.ly) * nx + (unsigned)gx;
    s.d1 = (unsigned)s.rgz * nxy + (unsigned)s.rgy * nx;
    s.d2 = nxy - (unsigned)b.e[1] * nx;
    s.li = tr * b.e[0] + tx;
    s.lstep = rg * b.e[0];
    return s;
}

// value of the current element (0 outside the volume), then advance a pass
template <bool CHECK>
__device__ __forceinline__ float stage_next(Stage& s, const float* __restrict__ vol, const VolDims& v, const Box& b)
{
    float val = 0.0f;
    // (CHECK false: the caller knows the box lies inside the volume)
    if (!CHECK || (s.xok && (unsigned)(b.o[1] + s.ly) < (unsigned)v.ny && (unsigned)(b.o[2] + s.lz) < (unsigned)v.nz))
        val = vol[s.gi];
    s.ly += s.rgy;
    const bool c = s.ly >= b.e[1];
    s.ly -= c ? b.e[1] : 0;
    s.lz += s.rgz + (c ? 1 : 0);
    s.gi += s.d1 + (c ? s.d2 : 0u);
    s.li += s.lstep;
    return val;
}

// element i of a box wider than 256 along x
__device__ __forceinline__ float element_value(const float* __restrict__ vol, const VolDims& v, const Box& b, int i)
{
    const float r0 = 1.0f / (float)b.e[0], r1 = 1.0f / (float)b.e[1];
    const int q = (int)__builtin_floorf(((float)i + 0.5f) * r0);
    const int lx = i - (int)__umul24(q, b.e[0]);
    const int lz = (int)__builtin_floorf(((float)q + 0.5f) * r1);
    const int ly = q - (int)__umul24(lz, b.e[1]);
    const int gx = b.o[0] + lx, gy = b.o[1] + ly, gz = b.o[2] + lz;
    float val = 0.0f;
    if ((unsigned)gx < (unsigned)v.nx && (unsigned)gy < (unsigned)v.ny && (unsigned)gz < (unsigned)v.nz)
        val = vol[(__umul24((unsigned)gz, (unsigned)v.ny) + (unsigned)gy) * (unsigned)v.nx + (unsigned)gx];
    return val;
}

template <bool CHECK = true>
__device__ __forceinline__ void load_box(float* box, const float* __restrict__ vol, const VolDims& v, const Box& b)
{
    if (b.e[0] > 256) {
        const int n = b.e[0] * b.e[1] * b.e[2];
        for (int i = threadIdx.x; i < n; i += blockDim.x) box[i] = element_value(vol, v, b, i);
        return;
    }
    Stage s = stage_of(b, v);
    if (!CHECK) s.xok = true;
    while (s.lz < b.e[2]) {
        const int li = s.li;
        box[li] = stage_next<CHECK>(s, vol, v, b);
    }
}

// the box lies inside the volume (no staged cell needs a bounds check)
__device__ __forceinline__ bool box_inside(const Box& b, const VolDims& v)
{
    return b.o[0] >= 0 && b.o[1] >= 0 && b.o[2] >= 0 && b.o[0] + b.e[0] <= v.nx && b.o[1] + b.e[1] <= v.ny &&
           b.o[2] + b.e[2] <= v.nz;
}

// Software-pipelined staging: the first PF passes of the next slab's box
// are loaded into registers while the current slab is sampled, then written
// to LDS; any further passes are read directly when the box is written.
template <int PF>
__device__ __forceinline__ void fetch_box(float (&r)[PF], const float* __restrict__ vol, const VolDims& v,
                                          const Box& b, bool on)
{
    if (on && b.e[0] <= 256) {
        Stage s = stage_of(b, v);
        if (box_inside(b, v)) {
#pragma unroll
            for (int m = 0; m < PF; ++m) {
                const bool row = s.lz < b.e[2];
                const float val = row ? stage_next<false>(s, vol, v, b) : 0.0f;
                r[m] = val;
            }
        } else {
#pragma unroll
            for (int m = 0; m < PF; ++m) {
                const bool row = s.lz < b.e[2];
                const float val = stage_next<true>(s, vol, v, b);
                r[m] = row ? val : 0.0f;
            }
        }
    } else {
#pragma unroll
        for (int m = 0; m < PF; ++m) r[m] = 0.0f;
    }
}

template <int PF>
__device__ __forceinline__ void put_box(float* box, const float (&r)[PF], const float* __restrict__ vol,
                                        const VolDims& v, const Box& b, bool on)
{
    if (!on) return;
    if (b.e[0] > 256) {
        load_box(box, vol, v, b);
        return;
    }
    Stage s = stage_of(b, v);
#pragma unroll
    for (int m = 0; m < PF; ++m) {
        if (s.lz < b.e[2]) box[s.li] = r[m];
        s.ly += s.rgy;
        const bool c = s.ly >= b.e[1];
        s.ly -= c ? b.e[1] : 0;
        s.lz += s.rgz + (c ? 1 : 0);
        s.gi += s.d1 + (c ? s.d2 : 0u);
        s.li += s.lstep;
    }
    if (box_inside(b, v)) {
        while (s.lz < b.e[2]) {
            const int li = s.li;
            box[li] = stage_next<false>(s, vol, v, b);
        }
    } else {
        while (s.lz < b.e[2]) {
            const int li = s.li;
            box[li] = stage_next<true>(s, vol, v, b);
        }
    }
}

// ------------------------------------------------------------------ Siddon
// The Siddon sum is taken one layer at a time along the tile's dominant
// axis a (a layer is one cell thick along a; the two other axes are b and
// c).  Inside a layer a ray whose direction has |d_b| and |d_c| below
// 0.99 |d_a| crosses at most one plane of b and one of c, so it passes
// through at most three cells; the three lengths follow from the two next
// crossing parameters by a min, a max and two clamps, and the three cells
// from which crossings fall inside the layer.  Every lane of a wave then
// does the same work per layer (no data-dependent branch), instead of one
// loop trip per crossing with the crossing axis chosen per lane.  The
// crossing parameters are the plane-by-plane walk's (plane q at q inv + c,
// FP32), so the lengths are that walk's, in the same cells.
//
// Two cases leave the three-cell form: a tile holding a ray steeper than
// 0.99 along b or c (it may cross two planes of one axis in a layer) and a
// ray whose path through a slab leaves the staged box (a box clipped to the
// LDS capacity).  Those lanes walk the layer plane by plane, reading cells
// outside the box from global memory.
__device__ __forceinline__ float sid_cell(const float* box, const float* __restrict__ vol, const VolDims& v,
                                          const Box& bx, int x, int y, int z)
{
    const int lx = x - bx.o[0], ly = y - bx.o[1], lz = z - bx.o[2];
    if ((unsigned)lx < (unsigned)bx.e[0] && (unsigned)ly < (unsigned)bx.e[1] && (unsigned)lz < (unsigned)bx.e[2])
        return box[(lz * bx.e[1] + ly) * bx.e[0] + lx];
    if ((unsigned)x < (unsigned)v.nx && (unsigned)y < (unsigned)v.ny && (unsigned)z < (unsigned)v.nz)
        return vol[(__umul24((unsigned)z, (unsigned)v.ny) + (unsigned)y) * (unsigned)v.nx + (unsigned)x];
    return 0.0f;
}

template <typename T>
__device__ __forceinline__ T pick3(int i, T v0, T v1, T v2)
{
    return i == 0 ? v0 : (i == 1 ? v1 : v2);
}

__device__ __forceinline__ SiddonAxis pick_axis(int i, const SiddonAxis& x, const SiddonAxis& y, const SiddonAxis& z)
{
    SiddonAxis r;
    r.inv = pick3(i, x.inv, y.inv, z.inv);
    r.c = pick3(i, x.c, y.c, z.c);
    r.step = pick3(i, x.step, y.step, z.step);
    return r;
}

// One ray's position in the layer walk: current parameter, end of the
// clipped ray, and per non-dominant axis the plane coordinate of the next
// crossing (an exact integer in FP32) with its parameter.
struct LayerRay {
    float acur, aend, qb, qc, anb, anc, acc;
};

// Plane-by-plane walk of one layer (cell k along a) up to parameter ae.
__device__ __forceinline__ void walk_layer(LayerRay& r, float ae, int k, int a, const SiddonAxis& B,
                                           const SiddonAxis& C, const float* box, const float* __restrict__ vol,
                                           const VolDims& v, const Box& bx)
{
    // at most two crossings of each of b and c fall inside one layer of a
    // ray that runs within 45 degrees of a (the tile's dominant axis); the
    // bound only caps the loop
    for (int it = 0; it < 8 && r.acur < ae; ++it) {
        const float an = fminf(fminf(r.anb, r.anc), ae);
        const int ib = (int)r.qb - (B.step > 0), ic = (int)r.qc - (C.step > 0);
        const int x = a == 0 ? k : ib, y = a == 1 ? k : (a == 0 ? ib : ic), z = a == 2 ? k : ic;
        r.acc = __builtin_fmaf(an - r.acur, sid_cell(box, vol, v, bx, x, y, z), r.acc);
        r.acur = an;
        if (an >= ae) break;
        if (r.anb <= r.anc) {
            r.qb += (float)B.step;
            r.anb = __builtin_fmaf(r.qb, B.inv, B.c);
        } else {
            r.qc += (float)C.step;
            r.anc = __builtin_fmaf(r.qc, C.inv, C.c);
        }
    }
    r.acur = ae;
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CTMI_FWD_SID_WAVES, 8))) k_forward_siddon(const float* __restrict__ vol, float* __restrict__ proj,
                                                        const ViewGeo* __restrict__ tab,
                                                        const ViewGeo64* __restrict__ tab64, int view0, TileMap m,
                                                        VolDims v, DetDims det)
{
    __shared__ float box[BOXCAP];
    __shared__ int sbox[SLABTAB][7];   // the first SLABTAB slabs' boxes (origin, extent, non-empty)
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
    float amin = a_lo, amax = a_hi;
    bool hit = slab_clip(ax, S[0], 0.0f, (float)v.nx, amin, amax);
    hit &= slab_clip(ay, S[1], 0.0f, (float)v.ny, amin, amax);
    hit &= slab_clip(az, S[2], 0.0f, (float)v.nz, amin, amax);
    const bool alive = active && hit && amin < amax;

    int a, dir;
    tile_axis(g, det, tu0, tv0, a, dir);
    const int b = a == 0 ? 1 : 0, c = a == 2 ? 1 : 2;
    const SiddonAxis A = pick_axis(a, ax, ay, az), B = pick_axis(b, ax, ay, az), C = pick_axis(c, ax, ay, az);
    const float Sa = pick3(a, S[0], S[1], S[2]), Da = pick3(a, d[0], d[1], d[2]);
    const float Sb = pick3(b, S[0], S[1], S[2]), Db = pick3(b, d[0], d[1], d[2]);
    const float Sc = pick3(c, S[0], S[1], S[2]), Dc = pick3(c, d[0], d[1], d[2]);
    const int na = pick3(a, v.nx, v.ny, v.nz), nb = pick3(b, v.nx, v.ny, v.nz), nc = pick3(c, v.nx, v.ny, v.nz);

    // a ray that runs against the tile's direction along a (only possible
    // at extreme fan angles) is walked plane by plane from global memory at
    // the end instead
    const bool odd = alive && A.step != dir;
    const bool lay = alive && !odd;
    LayerRay r;
    r.acc = 0.0f;
    r.acur = lay ? amin : 0.0f;
    r.aend = lay ? amax : 0.0f;
    {
        const int ib = ordered_cell(B, Sb, Db, amin, 0, nb), ic = ordered_cell(C, Sc, Dc, amin, 0, nc);
        r.qb = (float)(ib + (B.step > 0));
        r.qc = (float)(ic + (C.step > 0));
        // a parallel axis has inv = 0 and c = inf, so its crossings stay at inf
        r.anb = lay ? __builtin_fmaf(r.qb, B.inv, B.c) : CTMI_INF;
        r.anc = lay ? __builtin_fmaf(r.qc, C.inv, C.c) : CTMI_INF;
    }
    // the wave's layer range (cells along a that some lane's ray reaches)
    int klo = 0x7fffffff, khi = -1;
    if (lay) {
        const float p0 = __builtin_fmaf(amin, Da, Sa), p1 = __builtin_fmaf(amax, Da, Sa);
        klo = max((int)__builtin_floorf(fminf(p0, p1)) - 1, 0);
        khi = min((int)__builtin_floorf(fmaxf(p0, p1)) + 1, na - 1);
    }
    // the three-cell form needs every ray of the wave below 0.99 along b and c
    bool steep = lay && (fabsf(Db) > 0.99f * fabsf(Da) || fabsf(Dc) > 0.99f * fabsf(Da));
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        klo = min(klo, __shfl_xor(klo, off));
        khi = max(khi, __shfl_xor(khi, off));
    }
    // (the same in every lane now: keep them in scalar registers)
    klo = __builtin_amdgcn_readfirstlane(klo);
    khi = __builtin_amdgcn_readfirstlane(khi);
    const bool wave_steep = __any(steep);

    const int nslab = (na + SID_SLAB - 1) / SID_SLAB;
    const int clo[3] = {0, 0, 0}, chi[3] = {v.nx - 1, v.ny - 1, v.nz - 1};
    // the staged box of slab si (in the direction of travel): the cells
    // under the bundle, no margin (a ray whose walk rounds into a cell
    // outside, a corner ray within ulps of a plane, finds out below and
    // reads that slab plane by plane)
    auto slab_box = [&](int si, Box& bx) -> bool {
        const int s = dir > 0 ? si : nslab - 1 - si;
        const int c0 = s * SID_SLAB, c1 = min(c0 + SID_SLAB, na);   // cells [c0, c1) along a
        float blo[3], bhi[3];
        bundle_bounds(g, det, tu0, tv0, a, (float)c0, (float)c1, 0.0f, blo, bhi);
        int lo[3], hi[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lo[i] = (int)__builtin_floorf(fmaxf(blo[i], -4.0f));
            hi[i] = (int)__builtin_floorf(fminf(bhi[i], 1.0e7f));
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            lo[i] = i == a ? c0 : lo[i];
            hi[i] = i == a ? c1 - 1 : hi[i];
        }
        return make_box(lo, hi, clo, chi, a, bx);
    };
    // the first SLABTAB boxes are formed once, one slab per thread, instead
    // of by every wave at every slab
    if ((int)threadIdx.x < min(nslab, SLABTAB)) {
        Box bx;
        const bool ok = slab_box((int)threadIdx.x, bx);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            sbox[threadIdx.x][i] = bx.o[i];
            sbox[threadIdx.x][3 + i] = bx.e[i];
        }
        sbox[threadIdx.x][6] = ok ? 1 : 0;
    }
    __syncthreads();

    for (int si = 0; si < nslab; ++si) {
        const int s = dir > 0 ? si : nslab - 1 - si;
        const int c0 = s * SID_SLAB, c1 = min(c0 + SID_SLAB, na);   // cells [c0, c1) along a
        Box bx;
        bool ok;
        if (si < SLABTAB) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                bx.o[i] = sbox[si][i];
                bx.e[i] = sbox[si][3 + i];
            }
            ok = sbox[si][6] != 0;
        } else {
            ok = slab_box(si, bx);
        }
        if (!ok) continue;
        // the box is the same in every lane: scalar registers
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            bx.o[i] = __builtin_amdgcn_readfirstlane(bx.o[i]);
            bx.e[i] = __builtin_amdgcn_readfirstlane(bx.e[i]);
        }
        __syncthreads();
        load_box<false>(box, vol, v, bx);   // (clipped to the volume by make_box)
        __syncthreads();
        const int k0 = max(c0, klo), k1 = min(c1 - 1, khi);
        if (k0 > k1) continue;   // no ray of this wave reaches these layers

        // box strides (elements) and origins of the three axes
        const int st_a = pick3(a, 1, bx.e[0], bx.e[0] * bx.e[1]);
        const int st_b = pick3(b, 1, bx.e[0], bx.e[0] * bx.e[1]);
        const int st_c = pick3(c, 1, bx.e[0], bx.e[0] * bx.e[1]);
        const int oa = pick3(a, bx.o[0], bx.o[1], bx.o[2]);
        const int ob = pick3(b, bx.o[0], bx.o[1], bx.o[2]), eb = pick3(b, bx.e[0], bx.e[1], bx.e[2]);
        const int oc = pick3(c, bx.o[0], bx.o[1], bx.o[2]), ec = pick3(c, bx.e[0], bx.e[1], bx.e[2]);
        // does this ray's path through the slab stay inside the box?  Its
        // cells along b (and c) run monotonically from its current one to
        // the one it holds at the end of its stretch here, which
        // ordered_cell gives in the walk's crossing order; a ray with no
        // stretch here sits the slab out
        bool inbox = true, idle = true;
        int roff = 0;   // byte offset of the ray's (b, c) cell in a layer of the box
        {
            const float s0 = __builtin_fmaf((float)c0, A.inv, A.c), s1 = __builtin_fmaf((float)c1, A.inv, A.c);
            const float t0 = fmaxf(fminf(s0, s1), r.acur), t1 = fminf(fmaxf(s0, s1), r.aend);
            const int ib = (int)r.qb - (B.step > 0), ic = (int)r.qc - (C.step > 0);
            if (t0 < t1) {
                idle = false;
                const int ibe = ordered_cell(B, Sb, Db, t1, 0, nb), ice = ordered_cell(C, Sc, Dc, t1, 0, nc);
                inbox = min(ib, ibe) >= ob && max(ib, ibe) < ob + eb && min(ic, ice) >= oc && max(ic, ice) < oc + ec;
                roff = inbox ? 4 * ((ib - ob) * st_b + (ic - oc) * st_c) : 0;
            }
        }
        const int DB = 4 * B.step * st_b, DC = 4 * C.step * st_c;
        const char* boxb = (const char*)box;
        for (int kk = 0; kk <= k1 - k0; ++kk) {
            const int k = dir > 0 ? k0 + kk : k1 - kk;
            const float aa = __builtin_fmaf((float)(k + (dir > 0)), A.inv, A.c);   // exit plane of layer k
            const float ae = __builtin_amdgcn_fmed3f(aa, r.acur, r.aend);
            const int loff = 4 * (k - oa) * st_a;
            if (idle) {
            } else if (inbox && !wave_steep) {
                const bool cb = r.anb < ae, cc = r.anc < ae, bfirst = r.anb <= r.anc;
                const float t1 = __builtin_amdgcn_fmed3f(bfirst ? r.anb : r.anc, r.acur, ae);
                const float t2 = __builtin_amdgcn_fmed3f(bfirst ? r.anc : r.anb, r.acur, ae);
                const int db = cb ? DB : 0, dc = cc ? DC : 0;
                const int o0 = roff + loff;
                const float v0 = *(const float*)(boxb + o0);
                const float v1 = *(const float*)(boxb + o0 + (bfirst ? db : dc));
                const float v2 = *(const float*)(boxb + o0 + db + dc);
                r.acc = __builtin_fmaf(t1 - r.acur, v0, r.acc);
                r.acc = __builtin_fmaf(t2 - t1, v1, r.acc);
                r.acc = __builtin_fmaf(ae - t2, v2, r.acc);
                r.acur = ae;
                roff += db + dc;
                r.qb = cb ? r.qb + (float)B.step : r.qb;
                r.qc = cc ? r.qc + (float)C.step : r.qc;
                r.anb = __builtin_fmaf(r.qb, B.inv, B.c);
                r.anc = __builtin_fmaf(r.qc, C.inv, C.c);
            } else {
                walk_layer(r, ae, k, a, B, C, box, vol, v, bx);
                const int ib = (int)r.qb - (B.step > 0), ic = (int)r.qc - (C.step > 0);
                roff = 4 * ((ib - ob) * st_b + (ic - oc) * st_c);
            }
        }
    }
    if (odd) {
        // plane-by-plane walk over the whole ray from global memory
        int ix = ordered_cell(ax, S[0], d[0], amin, 0, v.nx);
        int iy = ordered_cell(ay, S[1], d[1], amin, 0, v.ny);
        int iz = ordered_cell(az, S[2], d[2], amin, 0, v.nz);
        float qx = (float)(ix + (ax.step > 0)), qy = (float)(iy + (ay.step > 0)), qz = (float)(iz + (az.step > 0));
        float anx = plane_alpha(ax, qx), any = plane_alpha(ay, qy), anz = plane_alpha(az, qz);
        float acur = amin;
        for (int left = v.nx + v.ny + v.nz + 3; left > 0; --left) {
            const float an = fminf(anx, fminf(any, anz));
            const float ae = fminf(an, amax);
            r.acc = __builtin_fmaf(fmaxf(ae - acur, 0.0f),
                                   vol[(__umul24((unsigned)iz, (unsigned)v.ny) + (unsigned)iy) * (unsigned)v.nx +
                                       (unsigned)ix],
                                   r.acc);
            if (an >= amax) break;
            acur = an;
            if (an == anx) {
                ix += ax.step;
                if ((unsigned)ix >= (unsigned)v.nx) break;
                qx += (float)ax.step;
                anx = plane_alpha(ax, qx);
            } else if (an == any) {
                iy += ay.step;
                if ((unsigned)iy >= (unsigned)v.ny) break;
                qy += (float)ay.step;
                any = plane_alpha(ay, qy);
            } else {
                iz += az.step;
                if ((unsigned)iz >= (unsigned)v.nz) break;
                qz += (float)az.step;
                anz = plane_alpha(az, qz);
            }
        }
    }
    if (active) proj[((int64_t)view * det.nv + iv) * det.nu + iu] = r.acc * L;
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
    __shared__ int sbox[SLABTAB][7];   // the first SLABTAB slabs' boxes (origin, extent, fits | clipped << 1)
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
    // the first SLABTAB boxes are formed once, one slab per thread, instead
    // of by every wave at every slab
    if ((int)threadIdx.x < min(nslab, SLABTAB)) {
        int A0, A1;
        Box bx;
        bool fits, clipped;
        slab_box((int)threadIdx.x, A0, A1, bx, fits, clipped);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            sbox[threadIdx.x][i] = bx.o[i];
            sbox[threadIdx.x][3 + i] = bx.e[i];
        }
        sbox[threadIdx.x][6] = (fits ? 1 : 0) | (clipped ? 2 : 0);
    }
    __syncthreads();
    auto slab_of = [&](int si, int& A0, int& A1, Box& b, bool& fits, bool& clipped) {
        if (si < SLABTAB) {
            const int s = dir > 0 ? si : nslab - 1 - si;
            A0 = s * SLAB - 1;
            A1 = A0 + SLAB;
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                b.o[i] = __builtin_amdgcn_readfirstlane(sbox[si][i]);
                b.e[i] = __builtin_amdgcn_readfirstlane(sbox[si][3 + i]);
            }
            const int f = __builtin_amdgcn_readfirstlane(sbox[si][6]);
            fits = (f & 1) != 0;
            clipped = (f & 2) != 0;
        } else {
            slab_box(si, A0, A1, b, fits, clipped);
        }
    };
    // the next slab's box is fetched into registers while this one is sampled
    constexpr int PF = CTMI_FWD_PF;
    float pf[PF];
    int nA0, nA1;
    Box nb;
    bool nfits, nclipped;
    slab_of(0, nA0, nA1, nb, nfits, nclipped);
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
            slab_of(si + 1, nA0, nA1, nb, nfits, nclipped);
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
            // samples k..kl by their offset j = k - kc from the ray's anchor, an
            // exact FP32 integer (interp_pos's position, without an int->float
            // conversion per sample).  Only a ray with samples here enters: its
            // offsets are below its sample count, far below 2^24, so the FP32
            // counter steps exactly and the loop ends.
            const float jl = (float)(kl - r.kc);
            for (float j = (float)(k - r.kc); k <= kl && j <= jl; j += 1.0f) {
                float p[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) p[i] = __builtin_fmaf(j, r.st[i], r.base[i]);
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
            k = max(k, kl + 1);
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
