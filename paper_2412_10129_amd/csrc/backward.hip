// Matched backprojectors: the exact transposes A^T of the Siddon and the
// interpolated forward projectors (needed by the Krylov methods of section
// 2.2.1, and as the gradient of the autograd operator).
//
// Voxel-driven by bricks: a workgroup owns one 16x16x8 brick of output voxels
// and accumulates it over every view of the call; each voxel has one writer
// in global memory and no global atomics are used.  For a group of views, the
// brick's detector footprints (bounding boxes of its projected corners) are
// enumerated in rounds of 256 (Siddon) or 512 (interpolated) pixels: each
// thread re-traces one or two pixels' rays inside the brick, with the same
// FP32 arithmetic as the forward kernel (shared helpers in ctmi_internal.h),
// and records them in an LDS ray table; the rays' work is cut into items of
// bounded size (a few cells or samples), numbered by a block scan, and
// processed round-robin so rays of different lengths keep every lane busy.
//
// Accumulation is in fixed point in LDS: FP32 LDS atomics are serialised
// on gfx950 (about 0.3 lane-ops per CU clock) while integer LDS atomics run
// 30-45x faster.  Views are taken in groups of 8.  The scale is chosen per
// round of rays (256 for Siddon, 512 interpolated) so that everything the
// round can add to one cell fits an int32: a Siddon ray adds at most one
// chord times |y| to a cell (it crosses a cell once); an interpolated ray at
// most K ds |y|, K the most samples of a ray inside a 2x2x2-voxel support;
// so the bound is that factor times the round's sum of |y|.  32-bit cells
// (about 1.4x faster atomics than 64-bit ones) hold the round's exact
// integer sum and are flushed after every round.  Flushes convert the integer sums (exact
// power-of-two scaling) into per-thread FP32 registers in a fixed order;
// integer addition is associative, so the result is bit-reproducible.
//
// The interpolated adjoint's rounds are latency-bound as much as
// arithmetic-bound (a round costs barriers, a block scan and a flush), so a
// round takes two rays per thread and needs three barriers.
#include "ctmi_internal.h"

#include <type_traits>

namespace ctmi {

namespace {

#ifndef CTMI_BWD_SID_CELLS
#define CTMI_BWD_SID_CELLS 16
#endif
#ifndef CTMI_BWD_INT_SAMPLES
#define CTMI_BWD_INT_SAMPLES 6
#endif
constexpr int BX = CTMI_BWD_BX, BY = CTMI_BWD_BY, BZ = CTMI_BWD_BZ;   // brick (voxels)
constexpr int NB = BX * BY * BZ;
constexpr int OWN = NB / 256;                     // voxels owned per thread
typedef unsigned long long u64;
typedef long long i64;

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
// [lo, hi] (per axis x, y, z): the pixel centres inside the bounding box of
// the 8 projected corners (the box's silhouette is their convex hull, so a
// ray through a centre outside it misses the box), widened by FOOT_EPS pixel
// against the FP32 rounding of the projection (about 1e-4 pixel; a ray that
// close to the box lies within 0.01 pixel of it, some 100 FP32 position
// rounding units, so a sample the FP32 walk might still place in the box is
// never left out), clamped to the detector.  Returns false if empty.
#ifndef CTMI_BWD_FOOT_EPS
#define CTMI_BWD_FOOT_EPS 0.01f
#endif
constexpr float FOOT_EPS = CTMI_BWD_FOOT_EPS;
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
    u0 = max((int)__builtin_ceilf(umin - FOOT_EPS), 0);
    v0 = max((int)__builtin_ceilf(vmin - FOOT_EPS), 0);
    u1 = min((int)__builtin_floorf(umax + FOOT_EPS), det.nu - 1);
    v1 = min((int)__builtin_floorf(vmax + FOOT_EPS), det.nv - 1);
    return u0 <= u1 && v0 <= v1;
}

// Exclusive prefix sum of one int per thread over a 256-thread block; returns
// this thread's offset and the block total.  `wsum` holds 4 ints of LDS.
__device__ __forceinline__ int block_scan(int v, int* wsum, int* total)
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        const int t = wsum[i];
        off += i < w ? t : 0;
        tot += t;
    }
    *total = tot;
    return off + x - v;
}

// Pixel of the current round taken by this thread (rounds cover 256
// consecutive footprint pixels).  With `spread` the thread index is
// bit-reversed: ray-table slots that sit next to each other (whose items run
// on neighbouring lanes) then hold pixels far apart on the detector.  The
// rays of adjacent pixels cross the same cells at the same steps, and LDS
// atomics of one instruction from several lanes to one address serialise
// (about 3x the cost of distinct addresses when 4 lanes share one).  The
// interpolated adjoint gains about 20% from it, the Siddon adjoint's layer
// walk about 3% (512^3 x 720: 580 -> 562 ms).
template <bool spread>
__device__ __forceinline__ int round_pixel(int p0)
{
    return p0 + (spread ? (int)(__builtin_bitreverse32(threadIdx.x) >> 24) : (int)threadIdx.x);
}
#ifndef CTMI_BWD_SPREAD
#define CTMI_BWD_SPREAD 1
#endif
#ifndef CTMI_BWD_SID_SPREAD
#define CTMI_BWD_SID_SPREAD 1
#endif

// Item -> ray map of one round: ray r owns items [pre[r], pre[r] + cnt).  The
// first MAPCAP items are looked up in a byte table written by the rays
// themselves; later ones (rare) by binary search over pre.
constexpr int MAPCAP = 4096;

__device__ __forceinline__ void fill_item_map(unsigned char* map, int off, int cnt)
{
    const int e = min(off + cnt, MAPCAP);
    for (int i = off; i < e; ++i) map[i] = (unsigned char)threadIdx.x;
}

// Sum of one float per thread over a 256-thread block, in a fixed order
// (deterministic).  `wsum` holds 4 floats of LDS; the call synchronises.
__device__ __forceinline__ float block_sum(float v, float* wsum)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) wsum[threadIdx.x >> 6] = v;
    __syncthreads();
    return (wsum[0] + wsum[1]) + (wsum[2] + wsum[3]);
}

// Largest r in [0, 255] with pre[r] <= it (pre non-decreasing).
__device__ __forceinline__ int owner(const int* pre, int it)
{
    int lo = 0, hi = 255;
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Fixed-point scale for one (brick, group of views) or one round: the
// exponent e of the largest power of two (up to exact powers of two) with
// 2^e cmax m <= 2^30, where cmax bounds a single contribution's matrix
// factor (one Siddon chord, or K samples of ds) and m > 0 is the group's
// largest |y| or the round's sum of |y| (finite values only).  Formed from
// the operands' exponents, so neither a product nor a quotient can
// overflow or underflow: with cmax = a 2^ec and m = b 2^em (a, b in
// [1/2, 1)), 2^(30 - ec - em) cmax m = 2^30 a b < 2^30, and one more
// power of two fits when a b < 1/2.  Contributions are scaled by 2^e and
// the integer sums by 2^-e with ldexp (exact), so the fixed point works at
// every magnitude of y that FP32 holds.
__device__ __forceinline__ int fixed_exp(float cmax, float m)
{
    int ec, em;
    const float a = __builtin_frexpf(cmax, &ec);
    const float b = __builtin_frexpf(m, &em);
    return 30 - ec - em + (a * b < 0.5f ? 1 : 0);
}

// |y| for finite y, 0 for NaN and infinities (those rays are handled by
// k_nonfinite after the accumulation)
__device__ __forceinline__ float finite_or_zero(float y)
{
    return __builtin_fabsf(y) <= 0x1.fffffep127f ? y : 0.0f;
}

// A contribution q (|q| <= 2^30 by the choice of scale) as a sign-extended
// 64-bit two's-complement integer (truncated toward zero: a bias below one
// unit).  The 64-bit accumulators then hold the exact sum of up to 2^33
// such terms.
__device__ __forceinline__ u64 to_fixed(float q)
{
    return (u64)(long long)(int)q;
}

// Views are processed in groups of GV: one fixed-point scale (from the max
// |y| over the group's footprints) and one flush per group, with the
// ray-setup rounds running over the group's combined footprint candidates.
// The group's footprints live in LDS.
#ifndef CTMI_BWD_GV
#define CTMI_BWD_GV 8
#endif
constexpr int GV = CTMI_BWD_GV;

struct GroupLds {
    int u0[GV], v0[GV], w[GV], pre[GV + 1];
    float rw[GV];   // 1 / w
    unsigned red;
};

// Footprints of views [k, k + n) (threads 0..n-1, one view each) and their
// candidate prefix; returns the candidate total (uniform).
__device__ __forceinline__ int make_group(GroupLds& G, const ViewGeo* __restrict__ tab, int view0, int k, int n,
                                          const float lo[3], const float hi[3], const DetDims& det)
{
    if ((int)threadIdx.x < GV) {
        const int g = threadIdx.x;
        int u0 = 0, u1 = -1, v0 = 0, v1 = -1;
        const bool ok = g < n && footprint(tab[view0 + k + g], lo, hi, det, u0, u1, v0, v1);
        G.u0[g] = u0;
        G.v0[g] = v0;
        G.w[g] = ok ? u1 - u0 + 1 : 1;
        G.rw[g] = 1.0f / (float)(ok ? u1 - u0 + 1 : 1);
        G.pre[g + 1] = ok ? (u1 - u0 + 1) * (v1 - v0 + 1) : 0;
    }
    if (threadIdx.x == 0) G.red = 0u;
    __syncthreads();
    if (threadIdx.x == 0) {
        G.pre[0] = 0;
        for (int g = 0; g < GV; ++g) G.pre[g + 1] += G.pre[g];
    }
    __syncthreads();
    return G.pre[GV];
}

// Candidate c of the group -> view g and pixel (iu, iv).  The row p / w is
// estimated in FP32 (p / w <= nv <= 2^20, so the estimate is within 1/4 of
// the quotient and its truncation off by at most one) and corrected with
// the exact remainder (w <= nu <= 4096 and the row fit __umul24).
__device__ __forceinline__ void group_pixel(const GroupLds& G, int c, int& g, int& iu, int& iv)
{
    g = 0;
#pragma unroll
    for (int i = 1; i < GV; ++i) g += c >= G.pre[i] ? 1 : 0;
    const int p = c - G.pre[g];
    const int w = G.w[g];
    int r = (int)((float)p * G.rw[g]);
    int rem = p - (int)__umul24((unsigned)r, (unsigned)w);
    if (rem < 0) {
        --r;
        rem += w;
    } else if (rem >= w) {
        ++r;
        rem -= w;
    }
    iv = G.v0[g] + r;
    iu = G.u0[g] + rem;
}

// Max |y| over the group's footprint pixels (block reduction).
__device__ __forceinline__ float group_max(GroupLds& G, const float* __restrict__ proj, const DetDims& det, int k,
                                           int total)
{
    float m = 0.0f;
    for (int c = threadIdx.x; c < total; c += blockDim.x) {
        int g, iu, iv;
        group_pixel(G, c, g, iu, iv);
        m = fmaxf(m, fabsf(finite_or_zero(proj[((int64_t)(k + g) * det.nv + iv) * det.nu + iu])));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmaxf(m, __shfl_xor(m, o, 64));
    if ((threadIdx.x & 63) == 0) atomicMax(&G.red, __float_as_uint(m));
    __syncthreads();
    return __uint_as_float(G.red);
}

// Add the view's fixed-point sums into the owned FP32 registers and clear
// those cells (voxel (lx, ly, lz) of the brick sits at
// ((lz + pad) * py + ly + pad) * px + lx + pad).  Each cell is read and
// cleared by the same thread; cells outside the brick that no flush reads
// are never cleared (they only collect discarded contributions).
template <typename Acc>
__device__ __forceinline__ void flush_view(Acc* acc, int px, int py, int pad, int e, float own[OWN])
{
#pragma unroll
    for (int m = 0; m < OWN; ++m) {
        const int i = threadIdx.x + 256 * m;
        const int lx = i % BX, ly = (i / BX) % BY, lz = i / (BX * BY);
        Acc* c = acc + ((lz + pad) * py + (ly + pad)) * px + (lx + pad);
        const Acc a = *c;
        *c = 0;
        own[m] += __builtin_ldexpf((float)(long long)a, -e);
    }
}

__device__ __forceinline__ void store_owned(float* __restrict__ vol, const float own[OWN], const VolDims& v, int x0,
                                            int y0, int z0, float beta)
{
#pragma unroll
    for (int m = 0; m < OWN; ++m) {
        const int i = threadIdx.x + 256 * m;
        const int gx = x0 + i % BX, gy = y0 + (i / BX) % BY, gz = z0 + i / (BX * BY);
        if (gx >= v.nx || gy >= v.ny || gz >= v.nz) continue;
        float* o = vol + ((int64_t)gz * v.ny + gy) * v.nx + gx;
        *o = beta == 0.0f ? own[m] : __builtin_fmaf(beta, *o, own[m]);
    }
}

// Accumulator cells: 32-bit (LDS atomics about 1.4x faster than 64-bit
// ones); the scale is chosen per round so that everything the round's rays
// can add to one cell fits (cmax sum_r |y_r|, cmax the most one ray adds to
// one cell per unit y: one chord for Siddon, whose rays cross a cell once;
// K samples of ds for the interpolated adjoint), the cells are flushed
// after every round, and contributions are rounded to nearest.  The Siddon
// adjoint's alternative (CTMI_BWD_SID_ACC32=0) keeps 64-bit cells with one
// scale per (brick, group) from the group's largest |y|, summed exactly over
// the group: 10 % slower with the layer walk (559 against 504 ms at 512^3 x
// 720; with the plane-by-plane walk it had been the faster one).
#ifndef CTMI_BWD_SID_ACC32
#define CTMI_BWD_SID_ACC32 1
#endif
constexpr bool SID_ACC32 = CTMI_BWD_SID_ACC32 != 0;
typedef std::conditional<SID_ACC32, int, u64>::type SAcc;

// floor(q + 1/2) as an int32 in one instruction (rintf costs a round and a
// convert); it differs from round-half-even only on exact ties
__device__ __forceinline__ int round_int(float q)
{
    int r;
    asm("v_cvt_rpi_i32_f32 %0, %1" : "=v"(r) : "v"(q));
    return r;
}
__device__ __forceinline__ void acc_add(int* a, float q) { atomicAdd(a, round_int(q)); }
__device__ __forceinline__ void acc_add(u64* a, float q) { atomicAdd(a, to_fixed(q)); }

constexpr int SID_CELLS = CTMI_BWD_SID_CELLS;   // dominant-axis cells per Siddon item

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

// An axis rebuilt from the (inv, c) that siddon_axis stored: inv has the
// sign of d, and is 0 (with c = inf) for a ray parallel to the planes
__device__ __forceinline__ SiddonAxis table_axis(float inv, float c)
{
    SiddonAxis r;
    r.inv = inv;
    r.c = c;
    r.step = inv > 0.0f ? 1 : (inv < 0.0f ? -1 : 0);
    return r;
}

// waves per SIMD the Siddon adjoint's registers are sized for: its 32-bit
// cells leave room for five workgroups per CU (31 KB of LDS each); 3 / 4 / 5
// measured 506 / 505 / 500 ms at 512^3 x 720 (five spill a few registers
// outside the walk)
#ifndef CTMI_BWD_SID_WAVES
#define CTMI_BWD_SID_WAVES 5
#endif
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CTMI_BWD_SID_WAVES, 8))) k_backward_siddon(const float* __restrict__ proj, float* __restrict__ vol,
                                                         const ViewGeo* __restrict__ tab,
                                                         const ViewGeo64* __restrict__ tab64, int view0, int nviews,
                                                         VolDims v, DetDims det, BrickMap m, float beta, float cmax)
{
    __shared__ SAcc acc[NB];
    __shared__ float t_S[3][256], t_d[3][256], t_inv[3][256], t_cc[3][256];
    __shared__ float t_a0[256], t_a1[256], t_y[256];
    __shared__ int t_c0[256], t_nc[256], t_pre[256];
    __shared__ unsigned char imap[MAPCAP];
    __shared__ int wsum[4];
    __shared__ float wsumf[4];
    __shared__ GroupLds G;
    for (int i = threadIdx.x; i < NB; i += blockDim.x) acc[i] = 0;
    float own[OWN];
#pragma unroll
    for (int i = 0; i < OWN; ++i) own[i] = 0.0f;
    int bx, by, bz;
    brick_origin(m, (int)blockIdx.x, bx, by, bz);
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
    const int x1 = min(x0 + BX, v.nx), y1 = min(y0 + BY, v.ny), z1 = min(z0 + BZ, v.nz);
    const float lo[3] = {x0 - 0.5f, y0 - 0.5f, z0 - 0.5f};   // cell box in voxel-centre coordinates
    const float hi[3] = {x1 - 0.5f, y1 - 0.5f, z1 - 0.5f};
    const int tid = threadIdx.x;

    for (int k = 0; k < nviews; k += GV) {
        const int ng = min(GV, nviews - k);
        __syncthreads();
        const int npx = make_group(G, tab, view0, k, ng, lo, hi, det);
        if (npx == 0) continue;
        // 64-bit cells: one scale per group from the largest |y| of its
        // footprints; 32-bit cells: one scale per round (below)
        const float maxy = SID_ACC32 ? 1.0f : group_max(G, proj, det, k, npx);
        if (!(maxy > 0.0f)) continue;
        int ex = SID_ACC32 ? 0 : fixed_exp(cmax, maxy);
        for (int p0 = 0; p0 < npx; p0 += 256) {
            const int p = round_pixel<CTMI_BWD_SID_SPREAD != 0>(p0);
            int cnt = 0;
            float yr = 0.0f, yl_ = 0.0f;   // this ray's y (finite, else 0), and its world length
            if (p < npx) {
                int gv, iu, iv;
                group_pixel(G, p, gv, iu, iv);
                const float* pk = proj + (int64_t)(k + gv) * det.nv * det.nu;
                float S[3], d[3], amin, amax;
                siddon_ray(tab64[view0 + k + gv], iu, iv, v, S, d, amin, amax);
                const SiddonAxis ax0 = siddon_axis(S[0], d[0]), ax1 = siddon_axis(S[1], d[1]),
                                 ax2 = siddon_axis(S[2], d[2]);
                bool hit = slab_clip(ax0, S[0], (float)x0, (float)x1, amin, amax);
                hit &= slab_clip(ax1, S[1], (float)y0, (float)y1, amin, amax);
                hit &= slab_clip(ax2, S[2], (float)z0, (float)z1, amin, amax);
                // the ray's dominant axis (largest |d|, never parallel to its planes);
                // selected by value so nothing is indexed at run time
                const int dom = (fabsf(d[0]) >= fabsf(d[1]) && fabsf(d[0]) >= fabsf(d[2])) ? 0
                                : (fabsf(d[1]) >= fabsf(d[2]) ? 1 : 2);
                if (hit && amin < amax) {
                    const float Sd = dom == 0 ? S[0] : (dom == 1 ? S[1] : S[2]);
                    const float dd = dom == 0 ? d[0] : (dom == 1 ? d[1] : d[2]);
                    const int sd = dom == 0 ? ax0.step : (dom == 1 ? ax1.step : ax2.step);
                    const int lod = dom == 0 ? x0 : (dom == 1 ? y0 : z0);
                    const int hid = dom == 0 ? x1 : (dom == 1 ? y1 : z1);
                    // dominant-axis cells from entry to exit
                    const int c0 = entry_cell(Sd, dd, amin, sd, lod, hid);
                    const int c1 = entry_cell(Sd, -dd, -amax, -sd, lod, hid);
                    const int nc = (c1 - c0) * sd + 1;
                    if (nc > 0) {
                        cnt = (nc + SID_CELLS - 1) / SID_CELLS;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            t_S[a][tid] = S[a];
                            t_d[a][tid] = d[a];
                        }
                        t_inv[0][tid] = ax0.inv;
                        t_inv[1][tid] = ax1.inv;
                        t_inv[2][tid] = ax2.inv;
                        t_cc[0][tid] = ax0.c;
                        t_cc[1][tid] = ax1.c;
                        t_cc[2][tid] = ax2.c;
                        t_a0[tid] = amin;
                        t_a1[tid] = amax;
                        t_c0[tid] = c0 * 4 + dom;
                        t_nc[tid] = nc;
                        yr = finite_or_zero(pk[(int64_t)iv * det.nu + iu]);
                        yl_ = world_length(d, v);
                    }
                }
            }
            int total;
            const int off = block_scan(cnt, wsum, &total);
            if (SID_ACC32) {
                // a ray crosses a cell once (items end on cell boundaries), so
                // one cell's round sum is at most cmax sum_r |y_r| (cmax: the
                // longest chord of a cell)
                const float ysum = block_sum(cnt > 0 ? fabsf(yr) : 0.0f, wsumf);
                if (!(ysum > 0.0f)) {
                    __syncthreads();
                    continue;
                }
                // (a sum of finite values overflows only when some |y| is near
                // FLT_MAX; 256 values of at most 2^128 bound it by 2^136)
                ex = ysum <= 0x1.fffffep127f ? fixed_exp(cmax, ysum) : fixed_exp(cmax, 0x1p127f) - 9;
            }
            // scaled before the length factor: |y 2^e| <= 2^30 / cmax
            if (cnt > 0) t_y[tid] = __builtin_ldexpf(yr, ex) * yl_;
            t_pre[tid] = off;
            fill_item_map(imap, off, cnt);
            __syncthreads();
            // items are taken round-robin (consecutive lanes on consecutive
            // items keep every lane's trip count at most SID_CELLS cells)
            for (int it = tid; it < total; it += 256) {
                const int r = it < MAPCAP ? (int)imap[it] : owner(t_pre, it);
                const int q = it - t_pre[r];
                const float S[3] = {t_S[0][r], t_S[1][r], t_S[2][r]};
                const float d[3] = {t_d[0][r], t_d[1][r], t_d[2][r]};
                // the ray's axes as its table row computed them (siddon_axis)
                const SiddonAxis ax = table_axis(t_inv[0][r], t_cc[0][r]);
                const SiddonAxis ay = table_axis(t_inv[1][r], t_cc[1][r]);
                const SiddonAxis az = table_axis(t_inv[2][r], t_cc[2][r]);
                const int dom = t_c0[r] & 3, c0 = t_c0[r] >> 2;
                const SiddonAxis ad = pick_axis(dom, ax, ay, az);
                const int nc = t_nc[r];
                const int cfirst = c0 + ad.step * q * SID_CELLS;
                const int nl = min(SID_CELLS, nc - q * SID_CELLS);   // dominant-axis cells (layers) of the item
                const int clast = cfirst + ad.step * (nl - 1);
                // the item spans dominant-axis cells cfirst..clast; its ends are
                // the planes the forward walk crosses there (same formula),
                // kept inside the ray's stretch in the brick: where the ray
                // leaves (or enters) through another face within a few ulps of
                // such a plane, the FP32 plane parameter can fall past the
                // stretch, and the walk must not cross that face
                const float a0r = t_a0[r], a1r = t_a1[r];
                const float astart = q == 0 ? a0r : fmaxf(plane_alpha(ad, (float)(cfirst + (ad.step < 0))), a0r);
                const float aend = (q * SID_CELLS + SID_CELLS >= nc)
                                       ? a1r
                                       : fminf(plane_alpha(ad, (float)(clast + (ad.step > 0))), a1r);
                const float yl = t_y[r];
                // the two other axes (b, c) of the ray
                const int b = dom == 0 ? 1 : 0, c = dom == 2 ? 1 : 2;
                const float Db = pick3(b, d[0], d[1], d[2]), Dc = pick3(c, d[0], d[1], d[2]);
                const float Dd = pick3(dom, d[0], d[1], d[2]);
                if (fabsf(Db) <= 0.99f * fabsf(Dd) && fabsf(Dc) <= 0.99f * fabsf(Dd)) {
                    // layer walk: within one dominant-axis cell the ray crosses at
                    // most one plane of b and one of c (it runs below 0.99 along
                    // both), so the cell's at most three segments follow from the
                    // two next crossing parameters (the forward kernel's form)
                    const SiddonAxis B = pick_axis(b, ax, ay, az), C = pick_axis(c, ax, ay, az);
                    const int ib = ordered_cell(B, pick3(b, S[0], S[1], S[2]), Db, astart, pick3(b, x0, y0, z0),
                                                pick3(b, x1, y1, z1));
                    const int ic = ordered_cell(C, pick3(c, S[0], S[1], S[2]), Dc, astart, pick3(c, x0, y0, z0),
                                                pick3(c, x1, y1, z1));
                    float qb = (float)(ib + (B.step > 0)), qc = (float)(ic + (C.step > 0));
                    // a parallel axis has inv = 0 and c = inf: its crossings stay at inf
                    float anb = __builtin_fmaf(qb, B.inv, B.c), anc = __builtin_fmaf(qc, C.inv, C.c);
                    const int ix = dom == 0 ? cfirst : (b == 0 ? ib : ic);
                    const int iy = dom == 1 ? cfirst : (dom == 0 ? ib : ic);
                    const int iz = dom == 2 ? cfirst : ic;
                    // cell offsets in bytes of the accumulator array
                    constexpr int E = (int)sizeof(SAcc);
                    int li = E * (int)(__umul24(__umul24(iz - z0, BY) + (iy - y0), BX) + (ix - x0));
                    const int SD = E * ad.step * pick3(dom, 1, BX, BX * BY);
                    const int DB = E * B.step * pick3(b, 1, BX, BX * BY), DC = E * C.step * pick3(c, 1, BX, BX * BY);
                    char* accb = (char*)acc;
                    float qa = (float)(cfirst + (ad.step > 0));   // exit plane of the current layer
                    const float fa = (float)ad.step, fb = (float)B.step, fc = (float)C.step;
                    // (an empty stretch, astart past aend by rounding, adds nothing)
                    float acur = fminf(astart, aend);
                    asm volatile("" ::"v"(yl), "v"(acur), "v"(aend), "v"(li));
                    for (int l = 0; l < nl; ++l) {
                        const float ae = __builtin_amdgcn_fmed3f(__builtin_fmaf(qa, ad.inv, ad.c), acur, aend);
                        const bool cb = anb < ae, cc = anc < ae, bfirst = anb <= anc;
                        const float t1 = __builtin_amdgcn_fmed3f(bfirst ? anb : anc, acur, ae);
                        const float t2 = __builtin_amdgcn_fmed3f(bfirst ? anc : anb, acur, ae);
                        const int db = cb ? DB : 0, dc = cc ? DC : 0;
                        const float s1 = t2 - t1, s2 = ae - t2;
                        acc_add((SAcc*)(accb + li), (t1 - acur) * yl);
                        if (s1 > 0.0f) acc_add((SAcc*)(accb + li + (bfirst ? db : dc)), s1 * yl);
                        if (s2 > 0.0f) acc_add((SAcc*)(accb + li + db + dc), s2 * yl);
                        acur = ae;
                        li += db + dc + SD;
                        qa += fa;
                        qb = cb ? qb + fb : qb;
                        qc = cc ? qc + fc : qc;
                        anb = __builtin_fmaf(qb, B.inv, B.c);
                        anc = __builtin_fmaf(qc, C.inv, C.c);
                    }
                    continue;
                }
                // a ray as steep along b or c as along its dominant axis (to 1 %)
                // may cross two planes of one axis in a layer: plane-by-plane walk
                int ix = ordered_cell(ax, S[0], d[0], astart, x0, x1);
                int iy = ordered_cell(ay, S[1], d[1], astart, y0, y1);
                int iz = ordered_cell(az, S[2], d[2], astart, z0, z1);
                if (dom == 0) ix = cfirst;
                else if (dom == 1) iy = cfirst;
                else iz = cfirst;
                float qx = (float)(ix + (ax.step > 0)), qy = (float)(iy + (ay.step > 0)), qz = (float)(iz + (az.step > 0));
                float anx = plane_alpha(ax, qx), any = plane_alpha(ay, qy), anz = plane_alpha(az, qz);
                int li = __umul24(__umul24(iz - z0, BY) + (iy - y0), BX) + (ix - x0);
                const int sx = ax.step, sy = ay.step * BX, sz = az.step * BX * BY;
                float acur = astart;
                const float fx = (float)ax.step, fy = (float)ay.step, fz = (float)az.step;
                asm volatile("" ::"v"(yl), "v"(acur), "v"(aend), "v"(li));
                // the crossing axis advances by selects, so lanes walking
                // different rays do not diverge over it
                for (int step = 0; step < BX + BY + BZ + 3; ++step) {
                    const float an = fminf(anx, fminf(any, anz));
                    const float ae = fminf(an, aend);
                    acc_add(&acc[li], fmaxf(ae - acur, 0.0f) * yl);
                    if (an >= aend) break;
                    acur = an;
                    const bool mx = an == anx, my = !mx && an == any, mz = !mx && !my;
                    ix += mx ? ax.step : 0;
                    iy += my ? ay.step : 0;
                    iz += mz ? az.step : 0;
                    if (ix < x0 || ix >= x1 || iy < y0 || iy >= y1 || iz < z0 || iz >= z1) break;
                    li += mx ? sx : (my ? sy : sz);
                    qx += mx ? fx : 0.0f;
                    qy += my ? fy : 0.0f;
                    qz += mz ? fz : 0.0f;
                    anx = mx ? plane_alpha(ax, qx) : anx;
                    any = my ? plane_alpha(ay, qy) : any;
                    anz = mz ? plane_alpha(az, qz) : anz;
                }
            }
            __syncthreads();
            if (SID_ACC32) {
                // 32-bit cells hold one round's sums (bounded by the scale)
                flush_view(acc, BX, BY, 0, ex, own);
                __syncthreads();
            }
        }
        if (!SID_ACC32) {
            flush_view(acc, BX, BY, 0, ex, own);
            __syncthreads();
        }
    }
    store_owned(vol, own, v, x0, y0, z0, beta);
}

constexpr int HX = BX + 2, HY = BY + 2, HZ = BZ + 2;   // interpolated accumulator: brick plus a one-voxel halo
constexpr int INT_SAMPLES = CTMI_BWD_INT_SAMPLES;  // samples per interpolated item

// Each interpolation sample is processed once, by the brick that holds its
// lower corner (the first brick of an axis also takes corners at -1, whose
// cell lies outside the volume).  Its upper corners may fall one voxel past
// the brick: those cells form the brick's upper shell, 553 cells in three
// faces (x = BX with y, z in [0, BY] x [0, BZ]; y = BY with x < BX; z = BZ
// with x < BX, y < BY), written to the plan's halo buffer and added to the
// neighbouring bricks' voxels by k_halo_add in a fixed order.
constexpr int HSX = (BY + 1) * (BZ + 1), HSY = BX * (BZ + 1), HSZ = BX * BY;
constexpr int HALO_SLOTS = HSX + HSY + HSZ;
constexpr int NH = (HALO_SLOTS + 255) / 256;   // shell cells per thread
static_assert(HALO_SLOTS == CTMI_HALO_SLOTS, "halo buffer size");

__device__ __forceinline__ void halo_slot(int h, int& lx, int& ly, int& lz)
{
    if (h < HSX) {
        lx = BX;
        ly = h % (BY + 1);
        lz = h / (BY + 1);
    } else if (h < HSX + HSY) {
        h -= HSX;
        lx = h % BX;
        ly = BY;
        lz = h / BX;
    } else {
        h -= HSX + HSY;
        lx = h % BX;
        ly = h / BX;
        lz = BZ;
    }
}

// shell cells -> per-thread FP32 registers, clearing them (accumulator
// origin at the brick corner minus one voxel)
template <typename Acc>
__device__ __forceinline__ void flush_shell(Acc* acc, int e, float hown[NH])
{
#pragma unroll
    for (int m = 0; m < NH; ++m) {
        const int h = threadIdx.x + 256 * m;
        if (h < HALO_SLOTS) {
            int lx, ly, lz;
            halo_slot(h, lx, ly, lz);
            Acc* c = acc + ((lz + 1) * HY + (ly + 1)) * HX + (lx + 1);
            const Acc a = *c;
            *c = 0;
            hown[m] += __builtin_ldexpf((float)(long long)a, -e);
        }
    }
}

// Rounds of the interpolated adjoint: RPT rays per thread, RAYS per round.
// Ray-table slot s = tid + 256 h (h < RPT) holds footprint pixel
// p0 + bitrev9(s), so slots next to each other (whose items run on
// neighbouring lanes) hold pixels far apart on the detector.  Item -> slot
// lookups go through a 16-bit map for the first IMAPCAP items of a round.
constexpr int RPT = 2, RAYS = 256 * RPT;
#ifndef CTMI_BWD_IMAPCAP
#define CTMI_BWD_IMAPCAP 4096
#endif
constexpr int IMAPCAP = CTMI_BWD_IMAPCAP;
static_assert(RAYS == 512, "slot permutation is a 9-bit reversal");

__device__ __forceinline__ int slot_pixel(int s)
{
    return CTMI_BWD_SPREAD ? (int)(__builtin_bitreverse32((unsigned)s) >> 23) : s;
}

// Largest slot r in [0, RAYS) with pre[r] <= it (pre non-decreasing).
__device__ __forceinline__ int owner_slot(const int* pre, int it)
{
    int lo = 0, hi = RAYS - 1;
#pragma unroll
    for (int st = 0; st < 9; ++st) {
        const int mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= it) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Inclusive scan of one int over a wave.
__device__ __forceinline__ int wave_scan(int x)
{
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x;
}

#ifndef CTMI_BWD_WAVES
#define CTMI_BWD_WAVES 4
#endif
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CTMI_BWD_WAVES, 8))) k_backward_interp(const float* __restrict__ proj, float* __restrict__ vol,
                                                         const ViewGeo* __restrict__ tab,
                                                         const ViewGeo64* __restrict__ tab64, int view0, int nviews,
                                                         VolDims v, DetDims det, BrickMap m, float beta, float ds,
                                                         float cmax, float* __restrict__ shell)
{
    // accumulator over voxels [b0 - 1, b1] per axis, so every sample scatters
    // to 8 fixed offsets without per-corner tests; the lower face only
    // receives corners outside the volume (first brick of an axis), the
    // upper shell goes to the neighbours
    __shared__ int acc[HX * HY * HZ];
    // ray table: (base, y) and (st, first sample | sample count << 16)
    __shared__ float4 t_a[RAYS], t_b[RAYS];
    __shared__ int t_pre[RAYS];
    __shared__ unsigned short imap[IMAPCAP];
    __shared__ int wsum[RPT][4];
    __shared__ float wsumf[4];
    __shared__ GroupLds G;
    for (int i = threadIdx.x; i < HX * HY * HZ; i += blockDim.x) acc[i] = 0;
    float own[OWN], hown[NH];
#pragma unroll
    for (int i = 0; i < OWN; ++i) own[i] = 0.0f;
#pragma unroll
    for (int i = 0; i < NH; ++i) hown[i] = 0.0f;
    int bx, by, bz;
    brick_origin(m, (int)blockIdx.x, bx, by, bz);
    const int x0 = bx * BX, y0 = by * BY, z0 = bz * BZ;
    const int x1 = min(x0 + BX, v.nx), y1 = min(y0 + BY, v.ny), z1 = min(z0 + BZ, v.nz);
    // the brick takes samples whose lower corner lies in [x0, x1) (from -1
    // for the first brick of an axis); their positions lie in [lo, hi)
    // (voxel-centre coordinates)
    const float lo[3] = {x0 > 0 ? (float)x0 : -1.0f, y0 > 0 ? (float)y0 : -1.0f, z0 > 0 ? (float)z0 : -1.0f};
    const float hi[3] = {(float)x1, (float)y1, (float)z1};
    // a sample's lower corner (floor of its position) must lie in
    // [lo, hi - 1] per axis; the accumulator's byte offset of corner c is
    // 4 ((c_z - z0 + 1) HX HY + (c_y - y0 + 1) HX + (c_x - x0 + 1)), formed
    // in FP32 (integers below 2^24)
    const float cmx = hi[0] - 1.0f, cmy = hi[1] - 1.0f, cmz = hi[2] - 1.0f;
    constexpr float AB = (float)sizeof(int);   // accumulator bytes per cell
    const float aoff =
        -AB * ((float)(z0 - 1) * (float)(HX * HY) + (float)(y0 - 1) * (float)HX + (float)(x0 - 1));
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    char* const accb = reinterpret_cast<char*>(acc);
    const float inv_ds = 1.0f / ds;

    for (int k = 0; k < nviews; k += GV) {
        const int ng = min(GV, nviews - k);
        __syncthreads();
        const int npx = make_group(G, tab, view0, k, ng, lo, hi, det);
        for (int p0 = 0; p0 < npx; p0 += RAYS) {
            // --- ray setup: RPT rays per thread
            int cnt[RPT];
            float ya = 0.0f;   // sum of |y| over this thread's rays
            float yr[RPT];
#pragma unroll
            for (int h = 0; h < RPT; ++h) {
                const int sl = tid + 256 * h;
                const int p = p0 + slot_pixel(sl);
                cnt[h] = 0;
                yr[h] = 0.0f;
                if (p < npx) {
                    int gv, iu, iv;
                    group_pixel(G, p, gv, iu, iv);
                    InterpRay ray;
                    if (interp_ray(tab64[view0 + k + gv], iu, iv, v, ds, inv_ds, ray)) {
                        // samples (relative to the anchor kc) inside the brick's
                        // box, widened by 1e-3 of a sample against the
                        // reciprocal's rounding, and by the samples within
                        // 2^-22 |face| of a face (|face| <= wface): a position
                        // that close may round onto either side of it, and for
                        // a ray nearly parallel to the face that span holds
                        // many samples (the smallest nonzero step bounds it on
                        // every axis).  A sample outside the box adds nothing
                        // (its weights are zeroed below), so widening only
                        // costs work, while a sample missed here would be lost.
                        float kmin = -CTMI_INF, kmax = CTMI_INF, imax = 0.0f;
                        bool inside = true;
#pragma unroll
                        for (int a = 0; a < 3; ++a) {
                            if (ray.st[a] != 0.0f) {
                                const float ia = ray.inv[a];
                                const float ka = (lo[a] - ray.base[a]) * ia, kb = (hi[a] - ray.base[a]) * ia;
                                kmin = fmaxf(kmin, fminf(ka, kb));
                                kmax = fminf(kmax, fmaxf(ka, kb));
                                imax = fmaxf(imax, fabsf(ia));
                            } else {
                                // constant coordinate: the loop's own test
                                const float f = __builtin_floorf(ray.base[a]);
                                inside &= f >= lo[a] && f <= hi[a] - 1.0f;
                            }
                        }
                        // (capped at 2^16 samples, more than a ray holds, so
                        // that the sample indices below stay in int range)
                        const float wface = 0x1p-22f * fmaxf(hi[0], fmaxf(hi[1], hi[2]));
                        const float wk = fminf(__builtin_fmaf(wface, imax, 1e-3f), 65536.0f);
                        if (inside && kmin < kmax + 2.0f * wk) {
                            const int ks = max(ray.k0, ray.kc + (int)__builtin_ceilf(kmin - wk));
                            const int ke = min(ray.k1, ray.kc + (int)__builtin_floorf(kmax + wk));
                            const int n = ke - ks + 1;
                            if (n > 0 && n < 65536) {
                                cnt[h] = (n + INT_SAMPLES - 1) / INT_SAMPLES;
                                // first sample relative to the anchor: |ks - kc| < 2^15
                                // because a ray has fewer than 2^15 samples in the
                                // volume (checked at plan creation)
                                const int jn = ((ks - ray.kc) & 0xFFFF) | (n << 16);
                                const float* pk = proj + (int64_t)(k + gv) * det.nv * det.nu;
                                yr[h] = pk[(int64_t)iv * det.nu + iu];
                                ya += fabsf(yr[h]);
                                t_a[sl] = make_float4(ray.base[0], ray.base[1], ray.base[2], 0.0f);
                                t_b[sl] = make_float4(ray.st[0], ray.st[1], ray.st[2], __int_as_float(jn));
                            }
                        }
                    }
                }
            }
            // --- one block pass: item offsets (exclusive scan over slots in
            // slot order) and the round's sum of |y| (fixed order)
            int inc[RPT];
#pragma unroll
            for (int h = 0; h < RPT; ++h) inc[h] = wave_scan(cnt[h]);
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) ya += __shfl_xor(ya, o, 64);
            if (lane == 63) {
#pragma unroll
                for (int h = 0; h < RPT; ++h) wsum[h][wid] = inc[h];
            }
            if (lane == 0) wsumf[wid] = ya;
            __syncthreads();
            float ysum = (wsumf[0] + wsumf[1]) + (wsumf[2] + wsumf[3]);
            if (!(ysum <= 0x1.fffffep127f)) {
                // a NaN or an infinity among the round's values (those rays
                // add nothing here; k_nonfinite marks their voxels), or a
                // finite sum past FLT_MAX: sum again over the finite values
                // (block-uniform branch)
                float yb = 0.0f;
#pragma unroll
                for (int h = 0; h < RPT; ++h) {
                    yr[h] = finite_or_zero(yr[h]);
                    yb += fabsf(yr[h]);
                }
#pragma unroll
                for (int o = 32; o > 0; o >>= 1) yb += __shfl_xor(yb, o, 64);
                __syncthreads();
                if (lane == 0) wsumf[wid] = yb;
                __syncthreads();
                ysum = (wsumf[0] + wsumf[1]) + (wsumf[2] + wsumf[3]);
            }
            if (!(ysum > 0.0f)) {
                // nothing to add: keep the LDS sums of this pass alive until
                // every thread has read them
                __syncthreads();
                continue;
            }
            int base = 0, off[RPT];
#pragma unroll
            for (int h = 0; h < RPT; ++h) {
                int before = 0, tot = 0;
#pragma unroll
                for (int w = 0; w < 4; ++w) {
                    const int t = wsum[h][w];
                    before += w < wid ? t : 0;
                    tot += t;
                }
                off[h] = base + before + inc[h] - cnt[h];
                base += tot;
            }
            const int total = base;
            // one cell's round sum is at most cmax sum_r |y_r| (cmax: K
            // samples of ds, K the most samples of one ray inside a
            // 2x2x2-voxel support)
            // (a sum of finite values can only overflow when some |y| is
            // near FLT_MAX; 512 values of at most 2^128 bound it by 2^137)
            const int ex = ysum <= 0x1.fffffep127f ? fixed_exp(cmax, ysum) : fixed_exp(cmax, 0x1p127f) - 10;
#pragma unroll
            for (int h = 0; h < RPT; ++h) {
                const int sl = tid + 256 * h;
                t_pre[sl] = off[h];
                if (cnt[h] > 0) {
                    // scaled before ds: |y 2^e| <= 2^30 / cmax and cmax >= ds
                    t_a[sl].w = __builtin_ldexpf(yr[h], ex) * ds;
                    const int e = min(off[h] + cnt[h], IMAPCAP);
                    for (int i = off[h]; i < e; ++i) imap[i] = (unsigned short)sl;
                }
            }
            __syncthreads();
            // --- items, taken round-robin: every lane runs at most
            // INT_SAMPLES samples per item, so the wave stays converged
            for (int it = tid; it < total; it += 256) {
                const int r = it < IMAPCAP ? (int)imap[it] : owner_slot(t_pre, it);
                const int q = it - t_pre[r];
                const float4 ta = t_a[r], tb = t_b[r];
                const int jn = __float_as_int(tb.w);
                const int j0 = (int)(int16_t)(uint16_t)(jn & 0xFFFF) + q * INT_SAMPLES;  // first sample
                const int cntq = min(INT_SAMPLES, (int)((unsigned)jn >> 16) - q * INT_SAMPLES);
                const float bxr = ta.x, byr = ta.y, bzr = ta.z, yv = ta.w;
                const float sxr = tb.x, syr = tb.y, szr = tb.z;
                // the ray's values must be in registers before the sample
                // loop, so that the loop never waits on its own atomics
                asm volatile("" ::"v"(bxr), "v"(byr), "v"(bzr), "v"(sxr), "v"(syr), "v"(szr), "v"(yv), "v"(j0),
                             "v"(cntq));
                // j runs over the item's samples as an exact FP32 integer
                const float jend = (float)(j0 + cntq);
                for (float j = (float)j0; j < jend; j += 1.0f) {
                    // same FP32 position as the forward kernel's sample k
                    const float px = __builtin_fmaf(j, sxr, bxr);
                    const float py = __builtin_fmaf(j, syr, byr);
                    const float pz = __builtin_fmaf(j, szr, bzr);
                    const float fx = __builtin_floorf(px), fy = __builtin_floorf(py), fz = __builtin_floorf(pz);
                    // corner clamped into the accumulator; a sample whose
                    // corner moved lies outside the box and adds 0
                    const float cx = __builtin_amdgcn_fmed3f(fx, lo[0], cmx);
                    const float cy = __builtin_amdgcn_fmed3f(fy, lo[1], cmy);
                    const float cz = __builtin_amdgcn_fmed3f(fz, lo[2], cmz);
                    const bool ok = cx == fx && cy == fy && cz == fz;
                    const int boff = (int)__builtin_fmaf(cz, AB * (float)(HX * HY),
                                                         __builtin_fmaf(cy, AB * (float)HX,
                                                                        __builtin_fmaf(cx, AB, aoff)));
                    const float ax_ = px - fx, ay_ = py - fy, az_ = pz - fz;
                    // trilinear weights times y, each pair split as (w - a w, a w)
                    const float yo = ok ? yv : 0.0f;
                    const float yz1 = az_ * yo, yz0 = yo - yz1;
                    const float w10 = ay_ * yz0, w00 = yz0 - w10;
                    const float w11 = ay_ * yz1, w01 = yz1 - w11;
                    const float u00 = ax_ * w00, u10 = ax_ * w10, u01 = ax_ * w01, u11 = ax_ * w11;
                    int* a0 = reinterpret_cast<int*>(accb + boff);
                    acc_add(a0, w00 - u00);
                    acc_add(a0 + 1, u00);
                    acc_add(a0 + HX, w10 - u10);
                    acc_add(a0 + HX + 1, u10);
                    acc_add(a0 + HX * HY, w01 - u01);
                    acc_add(a0 + HX * HY + 1, u01);
                    acc_add(a0 + HX * HY + HX, w11 - u11);
                    acc_add(a0 + HX * HY + HX + 1, u11);
                }
            }
            __syncthreads();
            // --- flush: 32-bit cells hold one round's sums (bounded by the
            // scale).  No barrier is needed after it: the next round's
            // atomics come after two more barriers, and nothing before them
            // touches the accumulator.
            flush_shell(acc, ex, hown);
            flush_view(acc, HX, HY, 1, ex, own);
        }
    }
    store_owned(vol, own, v, x0, y0, z0, beta);
    float* out = shell + (size_t)blockIdx.x * HALO_SLOTS;
#pragma unroll
    for (int m2 = 0; m2 < NH; ++m2) {
        const int h = threadIdx.x + 256 * m2;
        if (h < HALO_SLOTS) out[h] = hown[m2];
    }
}

// Adds the upper shells of the lower neighbour bricks to the voxels on each
// brick's lower faces, in a fixed order (x, y, z, xy, xz, yz, xyz
// neighbours).
__global__ void k_halo_add(float* __restrict__ vol, const float* __restrict__ shell, VolDims v, BrickMap m)
{
    const int64_t n = (int64_t)v.nx * v.ny * v.nz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int gx = (int)(i % v.nx);
    const int64_t r = i / v.nx;
    const int gy = (int)(r % v.ny), gz = (int)(r / v.ny);
    const int bx = gx / BX, by = gy / BY, bz = gz / BZ;
    const int lx = gx - bx * BX, ly = gy - by * BY, lz = gz - bz * BZ;
    if (lx != 0 && ly != 0 && lz != 0) return;
    auto cell = [&](int ex, int ey, int ez, int slot) {
        return shell[((size_t)((ez * m.nby + ey) * m.nbx + ex)) * HALO_SLOTS + slot];
    };
    const bool X = lx == 0 && bx > 0, Y = ly == 0 && by > 0, Z = lz == 0 && bz > 0;
    float add = 0.0f;
    if (X) add += cell(bx - 1, by, bz, ly + (BY + 1) * lz);
    if (Y) add += cell(bx, by - 1, bz, HSX + lx + BX * lz);
    if (Z) add += cell(bx, by, bz - 1, HSX + HSY + lx + BX * ly);
    if (X && Y) add += cell(bx - 1, by - 1, bz, BY + (BY + 1) * lz);
    if (X && Z) add += cell(bx - 1, by, bz - 1, ly + (BY + 1) * BZ);
    if (Y && Z) add += cell(bx, by - 1, bz - 1, HSX + lx + BX * BZ);
    if (X && Y && Z) add += cell(bx - 1, by - 1, bz - 1, BY + (BY + 1) * BZ);
    if (X || Y || Z) vol[i] += add;
}

// Non-finite projection values.  The adjoints above add finite values only
// (a NaN or infinite y_i counts as 0 there, which keeps the fixed-point
// scales finite); this pass then sets every voxel that such a ray reaches to
// NaN, since a_ij y_i is NaN or infinite there.  A voxel is reached when the
// Siddon walk gives it a piece of positive length, or when it is a corner of
// an interpolation sample inside the interpolant's support.  Rays are taken
// grid-stride, one per thread; a ray with a finite value costs one coalesced
// load.
template <bool SIDDON>
__global__ void __launch_bounds__(256) k_nonfinite(const float* __restrict__ proj, float* __restrict__ vol,
                                                   const ViewGeo64* __restrict__ tab64, int view0, int64_t nrays,
                                                   VolDims v, DetDims det, float ds, float inv_ds)
{
    const int64_t npix = (int64_t)det.nu * det.nv;
    const float qnan = __builtin_nanf("");
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nrays; i += (int64_t)gridDim.x * blockDim.x) {
        if (finite_or_zero(proj[i]) == proj[i]) continue;
        const int view = (int)(i / npix);
        const int pix = (int)(i - (int64_t)view * npix);
        const int iu = pix % det.nu, iv = pix / det.nu;
        const ViewGeo64& g = tab64[view0 + view];
        if (SIDDON) {
            float S[3], d[3], amin, amax;
            siddon_ray(g, iu, iv, v, S, d, amin, amax);
            const SiddonAxis ax = siddon_axis(S[0], d[0]), ay = siddon_axis(S[1], d[1]), az = siddon_axis(S[2], d[2]);
            bool hit = slab_clip(ax, S[0], 0.0f, (float)v.nx, amin, amax);
            hit &= slab_clip(ay, S[1], 0.0f, (float)v.ny, amin, amax);
            hit &= slab_clip(az, S[2], 0.0f, (float)v.nz, amin, amax);
            if (!hit || !(amin < amax)) continue;
            int ix = ordered_cell(ax, S[0], d[0], amin, 0, v.nx);
            int iy = ordered_cell(ay, S[1], d[1], amin, 0, v.ny);
            int iz = ordered_cell(az, S[2], d[2], amin, 0, v.nz);
            float anx = plane_alpha(ax, (float)(ix + (ax.step > 0)));
            float any = plane_alpha(ay, (float)(iy + (ay.step > 0)));
            float anz = plane_alpha(az, (float)(iz + (az.step > 0)));
            float acur = amin;
            for (int step = 0; step < v.nx + v.ny + v.nz + 3; ++step) {
                const float an = fminf(anx, fminf(any, anz));
                if (fminf(an, amax) > acur) vol[((int64_t)iz * v.ny + iy) * v.nx + ix] = qnan;
                if (an >= amax) break;
                acur = an;
                if (an == anx) {
                    ix += ax.step;
                    if (ix < 0 || ix >= v.nx) break;
                    anx = plane_alpha(ax, (float)(ix + (ax.step > 0)));
                } else if (an == any) {
                    iy += ay.step;
                    if (iy < 0 || iy >= v.ny) break;
                    any = plane_alpha(ay, (float)(iy + (ay.step > 0)));
                } else {
                    iz += az.step;
                    if (iz < 0 || iz >= v.nz) break;
                    anz = plane_alpha(az, (float)(iz + (az.step > 0)));
                }
            }
        } else {
            InterpRay r;
            if (!interp_ray(g, iu, iv, v, ds, inv_ds, r)) continue;
            for (int k = r.k0; k <= r.k1; ++k) {
                float p[3];
                interp_pos(r, k, p);
                if (!(p[0] > -1.0f && p[0] < (float)v.nx && p[1] > -1.0f && p[1] < (float)v.ny && p[2] > -1.0f &&
                      p[2] < (float)v.nz))
                    continue;
                const int fx = (int)__builtin_floorf(p[0]), fy = (int)__builtin_floorf(p[1]),
                          fz = (int)__builtin_floorf(p[2]);
#pragma unroll
                for (int c = 0; c < 8; ++c) {
                    const int cx = fx + (c & 1), cy = fy + ((c >> 1) & 1), cz = fz + (c >> 2);
                    if (cx >= 0 && cx < v.nx && cy >= 0 && cy < v.ny && cz >= 0 && cz < v.nz)
                        vol[((int64_t)cz * v.ny + cy) * v.nx + cx] = qnan;
                }
            }
        }
    }
}

BrickMap brick_map(const Plan& p)
{
    BrickMap m;
    m.nbx = (p.vol.nx + BX - 1) / BX;
    m.nby = (p.vol.ny + BY - 1) / BY;
    m.nbz = (p.vol.nz + BZ - 1) / BZ;
    return m;
}

template <bool SIDDON>
hipError_t launch_nonfinite(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews, hipStream_t s)
{
    const int64_t nrays = nviews * (int64_t)p.det.nu * p.det.nv;
    if (nrays == 0) return hipSuccess;
    const int64_t blocks = std::min<int64_t>((nrays + 255) / 256, 65536);
    hipLaunchKernelGGL(k_nonfinite<SIDDON>, dim3((unsigned)blocks), dim3(256), 0, s, proj, vol, p.d_views64,
                       (int)view0, nrays, p.vol, p.det, p.ds, 1.0f / p.ds);
    return hipGetLastError();
}

}  // namespace

int64_t adjoint_bricks(const Plan& p)
{
    const BrickMap m = brick_map(p);
    return (int64_t)m.nbx * m.nby * m.nbz;
}

size_t interp_adjoint_ws_bytes(const Plan& p) { return sizeof(float) * (size_t)adjoint_bricks(p) * HALO_SLOTS; }

hipError_t launch_backward_siddon(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                                  float beta, hipStream_t s)
{
    const BrickMap m = brick_map(p);
    const unsigned blocks = (unsigned)m.nbx * m.nby * m.nbz;
    hipLaunchKernelGGL(k_backward_siddon, dim3(blocks), dim3(256), 0, s, proj, vol, p.d_views, p.d_views64, (int)view0,
                       (int)nviews, p.vol, p.det, m, beta, SID_ACC32 ? p.round_siddon : p.entry_siddon);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_nonfinite<true>(p, proj, vol, view0, nviews, s);
}

hipError_t launch_backward_interp(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                                  float beta, float* shell, hipStream_t s)
{
    const BrickMap m = brick_map(p);
    const unsigned blocks = (unsigned)m.nbx * m.nby * m.nbz;
    hipLaunchKernelGGL(k_backward_interp, dim3(blocks), dim3(256), 0, s, proj, vol, p.d_views, p.d_views64, (int)view0,
                       (int)nviews, p.vol, p.det, m, beta, p.ds, p.round_interp, shell);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t n = (int64_t)p.vol.nx * p.vol.ny * p.vol.nz;
    hipLaunchKernelGGL(k_halo_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, vol, shell, p.vol, m);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_nonfinite<false>(p, proj, vol, view0, nviews, s);
}

}  // namespace ctmi
