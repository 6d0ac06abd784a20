// Kernels of the learned prior: a 3-D residual U-Net in BF16 with FP32
// accumulation, used plug-and-play inside CGLS.  The paper only says that
// trained networks call the projection operators; the network itself is
// the builder's choice (4 levels of 16/32/64/128 channels, 3x3x3 convs with
// ReLU, 2x2x2 average pooling, stride-2 2x2x2 transposed convs, skip
// concatenation, a 1x1x1 residual head).
//
// Layout: activations are channels-last BF16, [n][z][y][x][ld] with the
// tensor's channels at [0, C) of each voxel's ld-element row, so a channel
// concatenation is two (pointer, count, ld) operands and costs nothing.
// 3x3x3 weights are BF16 [cout][27][cin] with tap t = 9 kz + 3 ky + kx
// reading the input at (z + kz - 1, y + ky - 1, x + kx - 1).
//
// The 3x3x3 convolution is an implicit GEMM on the gfx950 BF16 MFMA
// (16x16x32, FP32 accumulators): D[co][voxel] = sum_k W[co][k] X[k][voxel]
// with k = (tap, ci).  A workgroup owns 2 x 8 x 16 output voxels and every
// output channel; input channels are staged 16 at a time as a halo brick in
// LDS (48-byte voxel stride: the sixteen 16-byte lane reads of a row hit
// disjoint banks), and one MFMA step covers two taps x 16 channels.  Weights
// stream from L1/L2 (they are small and shared by every workgroup).  The
// data gradient is the same kernel with flipped, transposed weights.
#include "ctmi_internal.h"

namespace ctmi {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef uint16_t u16;

__device__ __forceinline__ float bf2f(u16 h) { return __uint_as_float((uint32_t)h << 16); }

// FP32 -> BF16, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ u16 f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (u16)(u >> 16);
}

__device__ __forceinline__ bool bf_pos(u16 h) { return h != 0 && !(h & 0x8000u); }

__device__ __forceinline__ void unpack8(const uint4 q, float* f)
{
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        f[2 * i] = __uint_as_float(w[i] << 16);
        f[2 * i + 1] = __uint_as_float(w[i] & 0xFFFF0000u);
    }
}

__device__ __forceinline__ uint4 pack8(const float* f)
{
    uint4 q;
    q.x = (uint32_t)f2bf(f[0]) | ((uint32_t)f2bf(f[1]) << 16);
    q.y = (uint32_t)f2bf(f[2]) | ((uint32_t)f2bf(f[3]) << 16);
    q.z = (uint32_t)f2bf(f[4]) | ((uint32_t)f2bf(f[5]) << 16);
    q.w = (uint32_t)f2bf(f[6]) | ((uint32_t)f2bf(f[7]) << 16);
    return q;
}

__device__ __forceinline__ bf16x8 as_bf16x8(uint4 q)
{
    bf16x8 r;
    __builtin_memcpy(&r, &q, 16);
    return r;
}

// ------------------------------------------------------------------ conv3
constexpr int CX = 16, CY = 8, CZ = 2;               // output tile (x fastest)
constexpr int HX = CX + 2, HY = CY + 2, HZ = CZ + 2;  // halo brick
constexpr int HVOX = HX * HY * HZ;                    // 720
constexpr int VS = 24;                                // LDS voxel stride (u16): 16 ch + 8 pad

template <int NT>
__global__ __launch_bounds__(256) void k_conv3(UnetConv3 a)
{
    __shared__ __attribute__((aligned(16))) u16 xs[HVOX * VS];

    const int tiles_x = (a.w + CX - 1) / CX;
    const int x0 = (blockIdx.x % tiles_x) * CX;
    const int y0 = (blockIdx.x / tiles_x) * CY;
    const int z0 = blockIdx.y * CZ;
    const int nb = blockIdx.z;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int cin = a.c0 + a.c1;

    f32x4 acc[4][NT];
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int n = 0; n < NT; ++n) acc[r][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    const size_t plane = (size_t)a.h * a.w;
    const size_t vbase = (size_t)nb * a.d * plane;

    for (int cc = 0; cc < cin; cc += 16) {
        const u16* src;
        int ld;
        if (cc < a.c0) {
            src = a.in0 + cc;
            ld = a.ld0;
        } else {
            src = a.in1 + (cc - a.c0);
            ld = a.ld1;
        }
        __syncthreads();
        for (int i = tid; i < 2 * HVOX; i += 256) {
            const int hv = i >> 1, half = i & 1;
            const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint4 q = make_uint4(0, 0, 0, 0);
            if (gx >= 0 && gx < a.w && gy >= 0 && gy < a.h && gz >= 0 && gz < a.d)
                q = *reinterpret_cast<const uint4*>(src + (vbase + (size_t)gz * plane + (size_t)gy * a.w + gx) * ld +
                                                     half * 8);
            *reinterpret_cast<uint4*>(&xs[hv * VS + half * 8]) = q;
        }
        __syncthreads();

#pragma unroll 2
        for (int s = 0; s < 14; ++s) {
            const int tap = 2 * s + (g >> 1);
            const int ch = (g & 1) * 8;
            const bool valid = tap < 27;
            const int tz = tap / 9, ty = (tap / 3) % 3, tx = tap % 3;
            uint4 wf[NT];
#pragma unroll
            for (int n = 0; n < NT; ++n) {
                wf[n] = make_uint4(0, 0, 0, 0);
                if (valid)
                    wf[n] = *reinterpret_cast<const uint4*>(a.wt + ((size_t)(n * 16 + li) * 27 + tap) * cin + cc + ch);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int rr = wave * 4 + r;
                const int zl = rr >> 3, yl = rr & 7;
                const int hv = ((zl + tz) * HY + (yl + ty)) * HX + li + tx;
                uint4 xf = make_uint4(0, 0, 0, 0);
                if (valid) xf = *reinterpret_cast<const uint4*>(&xs[hv * VS + ch]);
                const bf16x8 xb = as_bf16x8(xf);
#pragma unroll
                for (int n = 0; n < NT; ++n)
                    acc[r][n] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(wf[n]), xb, acc[r][n], 0, 0, 0);
            }
        }
    }

    // epilogue: lane holds channels n*16 + 4g .. +3 of voxel (row, x0 + li)
    const int x = x0 + li;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int rr = wave * 4 + r;
        const int z = z0 + (rr >> 3), y = y0 + (rr & 7);
        if (x >= a.w || y >= a.h || z >= a.d) continue;
        const size_t vox = vbase + (size_t)z * plane + (size_t)y * a.w + x;
#pragma unroll
        for (int n = 0; n < NT; ++n) {
            const int co = n * 16 + 4 * g;
            float v[4] = {acc[r][n][0], acc[r][n][1], acc[r][n][2], acc[r][n][3]};
            if (a.bias) {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] += a.bias[co + e];
            }
            if (a.relu) {
#pragma unroll
                for (int e = 0; e < 4; ++e) v[e] = fmaxf(v[e], 0.0f);
            }
            if (a.mask) {
                const uint2 m = *reinterpret_cast<const uint2*>(a.mask + vox * a.ldm + co);
                if (!bf_pos((u16)(m.x & 0xFFFF))) v[0] = 0.0f;
                if (!bf_pos((u16)(m.x >> 16))) v[1] = 0.0f;
                if (!bf_pos((u16)(m.y & 0xFFFF))) v[2] = 0.0f;
                if (!bf_pos((u16)(m.y >> 16))) v[3] = 0.0f;
            }
            uint2 o;
            o.x = (uint32_t)f2bf(v[0]) | ((uint32_t)f2bf(v[1]) << 16);
            o.y = (uint32_t)f2bf(v[2]) | ((uint32_t)f2bf(v[3]) << 16);
            *reinterpret_cast<uint2*>(a.out + vox * a.ldo + co) = o;
        }
    }
}

// ------------------------------------------------------------ conv3 wgrad
// dW[co][t][ci] = sum_v dz[v][co] x[v + t][ci]: an MFMA GEMM with M = 16
// output channels, N = 16 input channels, K = voxels.  Both operands need 8
// consecutive voxels per lane, so the workgroup stages its 2 x 8 x 16 voxel
// tile transposed in LDS: dz as [co][voxel] and the input halo as three
// x-shifted copies [shift][ci][z][y][16] (one per kx, so every 8-voxel read
// is 16-byte aligned).  Wave w owns taps w, w + 4, ...; a workgroup owns
// one (co tile, ci tile) pair and a strided share of the voxel tiles, and
// writes its FP32 partial sums; a second kernel adds the partials in a
// fixed order.
constexpr int WG_DZS = 256 + 8;        // dz row stride (u16)
constexpr int WG_XROW = HZ * HY * 16;  // 640
constexpr int WG_XS = WG_XROW + 8;     // x ci-row stride (u16)

__global__ __launch_bounds__(256) void k_conv3_wgrad(UnetWgrad a)
{
    __shared__ __attribute__((aligned(16))) u16 dzs[16 * WG_DZS];
    __shared__ __attribute__((aligned(16))) u16 xsh[3 * 16 * WG_XS];

    const int ci_tiles = (a.c0 + a.c1) / 16;
    const int pair = blockIdx.x;
    const int cot = pair / ci_tiles, cit = pair % ci_tiles;
    const int split = blockIdx.y, nsplit = gridDim.y;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = lane >> 4, li = lane & 15;
    const int cin = a.c0 + a.c1;

    const u16* xsrc;
    int xld;
    if (cit * 16 < a.c0) {
        xsrc = a.in0 + cit * 16;
        xld = a.ld0;
    } else {
        xsrc = a.in1 + (cit * 16 - a.c0);
        xld = a.ld1;
    }
    const u16* dsrc = a.dz + cot * 16;

    const int tiles_x = (a.w + CX - 1) / CX, tiles_y = (a.h + CY - 1) / CY, tiles_z = (a.d + CZ - 1) / CZ;
    const int ntiles = tiles_x * tiles_y * tiles_z * a.n;
    const size_t plane = (size_t)a.h * a.w;

    f32x4 acc[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) acc[j] = f32x4{0.f, 0.f, 0.f, 0.f};

    for (int t = split; t < ntiles; t += nsplit) {
        int rem = t;
        const int tx_ = rem % tiles_x;
        rem /= tiles_x;
        const int ty_ = rem % tiles_y;
        rem /= tiles_y;
        const int tz_ = rem % tiles_z;
        const int nb = rem / tiles_z;
        const int x0 = tx_ * CX, y0 = ty_ * CY, z0 = tz_ * CZ;
        const size_t vbase = (size_t)nb * a.d * plane;

        __syncthreads();
        // dz tile: 256 voxels x 16 channels -> dzs[co][voxel]
        {
            const int v = tid;  // one voxel per thread
            const int xl = v & 15, yl = (v >> 4) & 7, zl = v >> 7;
            const int gx = x0 + xl, gy = y0 + yl, gz = z0 + zl;
            if (gx < a.w && gy < a.h && gz < a.d) {
                const u16* p = dsrc + (vbase + (size_t)gz * plane + (size_t)gy * a.w + gx) * a.ldz;
                const uint4 q0 = *reinterpret_cast<const uint4*>(p);
                const uint4 q1 = *reinterpret_cast<const uint4*>(p + 8);
                const uint32_t wd[8] = {q0.x, q0.y, q0.z, q0.w, q1.x, q1.y, q1.z, q1.w};
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    dzs[(2 * i) * WG_DZS + v] = (u16)(wd[i] & 0xFFFF);
                    dzs[(2 * i + 1) * WG_DZS + v] = (u16)(wd[i] >> 16);
                }
            } else {
#pragma unroll
                for (int i = 0; i < 16; ++i) dzs[i * WG_DZS + v] = 0;
            }
        }
        // input halo: 4 x 10 x 18 voxels x 16 channels -> three shifted copies
        for (int hv = tid; hv < HVOX; hv += 256) {
            const int hx = hv % HX, hy = (hv / HX) % HY, hz = hv / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            uint32_t wd[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            if (gx >= 0 && gx < a.w && gy >= 0 && gy < a.h && gz >= 0 && gz < a.d) {
                const u16* p = xsrc + (vbase + (size_t)gz * plane + (size_t)gy * a.w + gx) * xld;
                const uint4 q0 = *reinterpret_cast<const uint4*>(p);
                const uint4 q1 = *reinterpret_cast<const uint4*>(p + 8);
                wd[0] = q0.x; wd[1] = q0.y; wd[2] = q0.z; wd[3] = q0.w;
                wd[4] = q1.x; wd[5] = q1.y; wd[6] = q1.z; wd[7] = q1.w;
            }
            const int rowoff = (hz * HY + hy) * 16;
#pragma unroll
            for (int s = 0; s < 3; ++s) {
                const int j = hx - s;
                if (j < 0 || j >= 16) continue;
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    xsh[(s * 16 + 2 * i) * WG_XS + rowoff + j] = (u16)(wd[i] & 0xFFFF);
                    xsh[(s * 16 + 2 * i + 1) * WG_XS + rowoff + j] = (u16)(wd[i] >> 16);
                }
            }
        }
        __syncthreads();

        // K = 256 voxels in 8 steps of 32: lane group g takes row 2k + (g >> 1),
        // x-half (g & 1)
#pragma unroll 2
        for (int k = 0; k < 8; ++k) {
            const int rr = 2 * k + (g >> 1);
            const int xh = (g & 1) * 8;
            const int zl = rr >> 3, yl = rr & 7;
            const bf16x8 af = as_bf16x8(*reinterpret_cast<const uint4*>(&dzs[li * WG_DZS + rr * 16 + xh]));
#pragma unroll
            for (int j = 0; j < 7; ++j) {
                const int tap = wave + 4 * j;
                if (tap < 27) {
                    const int kz = tap / 9, ky = (tap / 3) % 3, kx = tap % 3;
                    const uint4 bq = *reinterpret_cast<const uint4*>(
                        &xsh[(kx * 16 + li) * WG_XS + ((zl + kz) * HY + (yl + ky)) * 16 + xh]);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af, as_bf16x8(bq), acc[j], 0, 0, 0);
                }
            }
        }
    }

    // partial[split][co][t][ci]: lane holds rows co = 4g + e, column ci = li
    float* part = a.partial + (size_t)split * a.cout * 27 * cin;
#pragma unroll
    for (int j = 0; j < 7; ++j) {
        const int tap = wave + 4 * j;
        if (tap >= 27) continue;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int co = cot * 16 + 4 * g + e;
            part[((size_t)co * 27 + tap) * cin + cit * 16 + li] = acc[j][e];
        }
    }
}

// out[i] = sum_s partial[s][i] (fixed order), FP32
// out[i] (+)= sum over k of partial[k][i]: a 256-thread block takes 32
// consecutive i and 8 lanes of splits (lane l sums the splits k = l mod 8 in
// order), then lane 0 adds the 8 lane sums in order: a fixed summation
// order, so the result is reproducible, with 8x the parallelism of one
// thread per i (the small layers have a few thousand weights over up to
// 1024 splits).
constexpr int SUM_E = 32, SUM_L = 8;
__global__ __launch_bounds__(256) void k_sum_partials(const float* __restrict__ partial, int nsplit, int64_t n,
                                                      float* __restrict__ out, int accumulate)
{
    __shared__ float red[SUM_L][SUM_E];
    const int e = threadIdx.x % SUM_E, l = threadIdx.x / SUM_E;
    const int64_t i = (int64_t)blockIdx.x * SUM_E + e;
    float s = 0.0f;
    if (i < n)
        for (int k = l; k < nsplit; k += SUM_L) s += partial[(size_t)k * n + i];
    red[l][e] = s;
    __syncthreads();
    if (l == 0 && i < n) {
        float t = red[0][e];
#pragma unroll
        for (int m = 1; m < SUM_L; ++m) t += red[m][e];
        out[i] = accumulate ? out[i] + t : t;
    }
}

// per-block channel sums of a BF16 tensor: partial[block][c] (FP32)
__global__ __launch_bounds__(256) void k_channel_sums(const u16* __restrict__ t, int ld, int c, int64_t nvox,
                                                      float* __restrict__ partial)
{
    __shared__ float red[256];
    // thread = (voxel lane vl, channel group of 8 cg); 256 / (c / 8) voxel lanes
    const int groups = c / 8;
    const int lanes = 256 / groups;
    const int tid = threadIdx.x;
    const int cg = tid % groups, vl = tid / groups;
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (vl < lanes) {
        for (int64_t v = (int64_t)blockIdx.x * lanes + vl; v < nvox; v += (int64_t)gridDim.x * lanes) {
            float f[8];
            unpack8(*reinterpret_cast<const uint4*>(t + v * ld + cg * 8), f);
#pragma unroll
            for (int i = 0; i < 8; ++i) s[i] += f[i];
        }
    }
    for (int i = 0; i < 8; ++i) {
        red[tid] = (vl < lanes) ? s[i] : 0.0f;
        __syncthreads();
        if (tid < groups) {
            float tot = 0.0f;
            for (int l = 0; l < lanes; ++l) tot += red[l * groups + tid];
            partial[(size_t)blockIdx.x * c + tid * 8 + i] = tot;
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ misc
// x (FP32, one channel) -> BF16 [v][16] with channel 0 = x, others 0: the
// first convolution then runs on the same MFMA kernel
__global__ void k_pack_input(const float* __restrict__ x, int64_t nvox, u16* __restrict__ out)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    uint4* o = reinterpret_cast<uint4*>(out + v * 16);
    o[0] = make_uint4((uint32_t)f2bf(x[v]), 0, 0, 0);
    o[1] = make_uint4(0, 0, 0, 0);
}

// 2x2x2 average pooling, 8 channels per thread
__global__ void k_pool2(const u16* __restrict__ in, int ldi, int n, int d, int h, int w, int c, u16* __restrict__ out,
                        int ldo)
{
    const int groups = c / 8;
    const int64_t total = (int64_t)n * d * h * w * groups;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int cg = (int)(i % groups);
    int64_t v = i / groups;
    const int x = (int)(v % w);
    v /= w;
    const int y = (int)(v % h);
    v /= h;
    const int z = (int)(v % d);
    const int nb = (int)(v / d);
    float s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int k = 0; k < 8; ++k) {
        const int zz = 2 * z + (k >> 2), yy = 2 * y + ((k >> 1) & 1), xx = 2 * x + (k & 1);
        const size_t fv = (((size_t)nb * 2 * d + zz) * 2 * h + yy) * 2 * w + xx;
        float f[8];
        unpack8(*reinterpret_cast<const uint4*>(in + fv * ldi + cg * 8), f);
#pragma unroll
        for (int e = 0; e < 8; ++e) s[e] += f[e];
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) s[e] *= 0.125f;
    const size_t cv = (((size_t)nb * d + z) * h + y) * w + x;
    *reinterpret_cast<uint4*>(out + cv * ldo + cg * 8) = pack8(s);
}

// gradient at a skip tensor e (fine grid) that feeds both a pooling and a
// concatenation: dz = mask(e) * (dp[parent] / 8 + dcat), rounded to BF16
__global__ void k_skip_grad(const u16* __restrict__ e, int lde, const u16* __restrict__ dp, int ldp,
                            const u16* __restrict__ dcat, int ldc, int n, int d, int h, int w, int c,
                            u16* __restrict__ out, int ldo)
{
    const int groups = c / 8;
    const int64_t total = (int64_t)n * d * h * w * groups;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int cg = (int)(i % groups);
    int64_t v = i / groups;
    const int x = (int)(v % w);
    v /= w;
    const int y = (int)(v % h);
    v /= h;
    const int z = (int)(v % d);
    const int nb = (int)(v / d);
    const size_t fv = (((size_t)nb * d + z) * h + y) * w + x;
    const size_t pv = (((size_t)nb * (d / 2) + z / 2) * (h / 2) + y / 2) * (w / 2) + x / 2;
    float fe[8], fp[8], fc[8];
    const uint4 qe = *reinterpret_cast<const uint4*>(e + fv * lde + cg * 8);
    unpack8(*reinterpret_cast<const uint4*>(dp + pv * ldp + cg * 8), fp);
    unpack8(*reinterpret_cast<const uint4*>(dcat + fv * ldc + cg * 8), fc);
    unpack8(qe, fe);
    float o[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) o[k] = (fe[k] > 0.0f) ? fp[k] * 0.125f + fc[k] : 0.0f;
    *reinterpret_cast<uint4*>(out + fv * ldo + cg * 8) = pack8(o);
}

// stride-2 2x2x2 transposed convolution: out[2v + s][co] =
// bf16(b[co] + sum_ci x[v][ci] w[co][s][ci]); thread = (fine voxel, 8 co)
__global__ void k_up2(const u16* __restrict__ x, int ldx, int cin, const u16* __restrict__ wt,
                      const float* __restrict__ bias, int cout, int n, int d, int h, int w, u16* __restrict__ out,
                      int ldo)
{
    const int groups = cout / 8;
    const int D = 2 * d, H = 2 * h, W = 2 * w;
    const int64_t total = (int64_t)n * D * H * W * groups;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int cg = (int)(i % groups);
    int64_t v = i / groups;
    const int X = (int)(v % W);
    v /= W;
    const int Y = (int)(v % H);
    v /= H;
    const int Z = (int)(v % D);
    const int nb = (int)(v / D);
    const int s = ((Z & 1) << 2) | ((Y & 1) << 1) | (X & 1);
    const size_t cv = (((size_t)nb * d + (Z >> 1)) * h + (Y >> 1)) * w + (X >> 1);
    float acc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = bias ? bias[cg * 8 + e] : 0.0f;
    const u16* xp = x + cv * ldx;
    for (int c8 = 0; c8 < cin; c8 += 8) {
        float fx[8];
        unpack8(*reinterpret_cast<const uint4*>(xp + c8), fx);
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float fw[8];
            unpack8(*reinterpret_cast<const uint4*>(wt + ((size_t)(cg * 8 + e) * 8 + s) * cin + c8), fw);
#pragma unroll
            for (int k = 0; k < 8; ++k) acc[e] = fmaf(fx[k], fw[k], acc[e]);
        }
    }
    const size_t fv = (((size_t)nb * D + Z) * H + Y) * W + X;
    *reinterpret_cast<uint4*>(out + fv * ldo + cg * 8) = pack8(acc);
}

// The same transposed convolution on the BF16 MFMA (16x16x32, FP32
// accumulators), for cin a multiple of 32 and cout of 16 * NT: per
// sub-position s, D_s[co][v] = sum_ci W[co][s][ci] X[ci][v] is a GEMM with
// M = cout, N = coarse voxels, K = cin.  A wave owns 16 consecutive coarse
// voxels (the N columns; lane li reads 8 consecutive channels of voxel
// v0 + li, a 16-byte load from the channels-last row) and computes all eight
// sub-positions and all output channels, so every input row is read once;
// the weights (at most 64 x 8 x 128 BF16) come through L1/L2.  Lane
// (li, g) ends with channels 16 nt + 4 g .. + 3 of fine voxel 2 v + s.
template <int NT>
__global__ __launch_bounds__(256) void k_up2_mfma(const u16* __restrict__ x, int ldx, int cin,
                                                  const u16* __restrict__ wt, const float* __restrict__ bias, int n,
                                                  int d, int h, int w, u16* __restrict__ out, int ldo)
{
    const int lane = threadIdx.x & 63, g = lane >> 4, li = lane & 15;
    const int64_t nvox = (int64_t)n * d * h * w;
    const int64_t v0 = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * 16;
    if (v0 >= nvox) return;   // uniform over the wave
    const int64_t v = v0 + li;
    const bool vok = v < nvox;
    const u16* xr = x + (vok ? v : v0) * ldx + 8 * g;
    int64_t r = vok ? v : v0;
    const int cx = (int)(r % w);
    r /= w;
    const int cy = (int)(r % h);
    r /= h;
    const int cz = (int)(r % d);
    const int nb = (int)(r / d);
    const int D = 2 * d, H = 2 * h, W = 2 * w;
    // sub-positions one at a time (the input row stays in L1 between them)
    for (int s = 0; s < 8; ++s) {
        f32x4 acc[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
        for (int kc = 0; kc < cin; kc += 32) {
            const bf16x8 xb = as_bf16x8(vok ? *reinterpret_cast<const uint4*>(xr + kc) : make_uint4(0, 0, 0, 0));
#pragma unroll
            for (int nt = 0; nt < NT; ++nt) {
                const uint4 wf =
                    *reinterpret_cast<const uint4*>(wt + ((size_t)(nt * 16 + li) * 8 + s) * cin + kc + 8 * g);
                acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(wf), xb, acc[nt], 0, 0, 0);
            }
        }
        // The accumulators are read right after the last MFMA; the compiler
        // left too few wait states there (the first two of each four read
        // stale values), so 24 explicit ones are placed between the MFMAs
        // that define them and the reads, pinned by in/out operands.
        if constexpr (NT == 1)
            asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" : "+a"(acc[0]));
        else if constexpr (NT == 2)
            asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" : "+a"(acc[0]), "+a"(acc[1]));
        else
            asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7"
                         : "+a"(acc[0]), "+a"(acc[1]), "+a"(acc[2]), "+a"(acc[3]));
        if (!vok) continue;
        const int Z = 2 * cz + (s >> 2), Y = 2 * cy + ((s >> 1) & 1), X = 2 * cx + (s & 1);
        const size_t fv = (((size_t)nb * D + Z) * H + Y) * W + X;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int co = nt * 16 + 4 * g;
            float o[4] = {acc[nt][0], acc[nt][1], acc[nt][2], acc[nt][3]};
            if (bias) {
#pragma unroll
                for (int e = 0; e < 4; ++e) o[e] += bias[co + e];
            }
            uint2 q;
            q.x = (uint32_t)f2bf(o[0]) | ((uint32_t)f2bf(o[1]) << 16);
            q.y = (uint32_t)f2bf(o[2]) | ((uint32_t)f2bf(o[3]) << 16);
            *reinterpret_cast<uint2*>(out + fv * ldo + co) = q;
        }
    }
}

// data gradient of up2 with the ReLU mask of its input:
// dx[v][ci] = bf16(mask(below[v][ci]) sum_s sum_co g[2v + s][co] w[co][s][ci])
__global__ void k_up2_dgrad(const u16* __restrict__ gr, int ldg, int cout, const u16* __restrict__ wt, int cin,
                            const u16* __restrict__ below, int ldb, int n, int d, int h, int w, u16* __restrict__ out,
                            int ldo)
{
    const int groups = cin / 8;
    const int64_t total = (int64_t)n * d * h * w * groups;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int cg = (int)(i % groups);
    int64_t v = i / groups;
    const int x = (int)(v % w);
    v /= w;
    const int y = (int)(v % h);
    v /= h;
    const int z = (int)(v % d);
    const int nb = (int)(v / d);
    float acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int s = 0; s < 8; ++s) {
        const int Z = 2 * z + (s >> 2), Y = 2 * y + ((s >> 1) & 1), X = 2 * x + (s & 1);
        const size_t fv = (((size_t)nb * 2 * d + Z) * 2 * h + Y) * 2 * w + X;
        const u16* gp = gr + fv * ldg;
        for (int c8 = 0; c8 < cout; c8 += 8) {
            float fg[8];
            unpack8(*reinterpret_cast<const uint4*>(gp + c8), fg);
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                float fw[8];
                unpack8(*reinterpret_cast<const uint4*>(wt + ((size_t)(c8 + e) * 8 + s) * cin + cg * 8), fw);
#pragma unroll
                for (int k = 0; k < 8; ++k) acc[k] = fmaf(fg[e], fw[k], acc[k]);
            }
        }
    }
    const size_t cv = (((size_t)nb * d + z) * h + y) * w + x;
    if (below) {
        float fb[8];
        unpack8(*reinterpret_cast<const uint4*>(below + cv * ldb + cg * 8), fb);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            if (!(fb[k] > 0.0f)) acc[k] = 0.0f;
    }
    *reinterpret_cast<uint4*>(out + cv * ldo + cg * 8) = pack8(acc);
}

// The same data gradient on the MFMA: D[ci][v] = sum_k W'[ci][k] G[k][v]
// with k = s cout + co, W'[ci][s cout + co] = w[co][s][ci] and G[k][v] =
// g[2v + s][co].  A wave owns 2 x 16 coarse voxels (B columns: lane li
// reads 8 consecutive co of fine voxel 2v + s, one 16-byte load); the
// workgroup stages each 32-wide k chunk of W' transposed in LDS ([ci][32],
// one 16-byte A fragment per lane and ci tile).  Lane (li, g) ends with
// ci = 16 nt + 4 g .. + 3 of voxel v0 + li.
#ifndef CTMI_UP2_DGRAD_MFMA
#define CTMI_UP2_DGRAD_MFMA 1
#endif
constexpr int UPD_VG = 2;   // 16-voxel groups per wave
template <int NT>
__global__ __launch_bounds__(256) void k_up2_dgrad_mfma(const u16* __restrict__ gr, int ldg, int cout,
                                                        const u16* __restrict__ wt, const u16* __restrict__ below,
                                                        int ldb, int n, int d, int h, int w, u16* __restrict__ out,
                                                        int ldo)
{
    constexpr int CIN = 16 * NT, WS = 40;   // LDS row stride (u16): 32 k + 8 pad
    __shared__ __attribute__((aligned(16))) u16 wl[CIN * WS];
    const int lane = threadIdx.x & 63, g = lane >> 4, li = lane & 15;
    const int64_t nvox = (int64_t)n * d * h * w;
    const int64_t vw = ((int64_t)blockIdx.x * 4 + (threadIdx.x >> 6)) * (16 * UPD_VG);   // the wave's first voxel
    const int D2 = 2 * d, H2 = 2 * h, W2 = 2 * w;
    int64_t fb[UPD_VG];   // fine index of sub-position 0 of each group's voxel
    bool vok[UPD_VG];
#pragma unroll
    for (int q = 0; q < UPD_VG; ++q) {
        const int64_t v = vw + 16 * q + li;
        vok[q] = v < nvox;
        int64_t r = vok[q] ? v : 0;
        const int cx = (int)(r % w);
        r /= w;
        const int cy = (int)(r % h);
        r /= h;
        const int cz = (int)(r % d);
        const int nb = (int)(r / d);
        fb[q] = (((int64_t)nb * D2 + 2 * cz) * H2 + 2 * cy) * W2 + 2 * cx;
    }
    f32x4 acc[UPD_VG][NT];
#pragma unroll
    for (int q = 0; q < UPD_VG; ++q)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) acc[q][nt] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int K = 8 * cout;
    for (int kc = 0; kc < K; kc += 32) {
        __syncthreads();   // the previous chunk's fragments have been read
        for (int i = threadIdx.x; i < CIN * 32; i += 256) {
            const int ci = i % CIN, kk = i / CIN;   // consecutive threads read consecutive ci
            const int k = kc + kk, s = k / cout, co = k - s * cout;
            wl[ci * WS + kk] = wt[((size_t)co * 8 + s) * CIN + ci];
        }
        __syncthreads();
        const int k = kc + 8 * g, s = k / cout, co0 = k - s * cout;
        const int64_t so = ((int64_t)(s >> 2) * H2 + ((s >> 1) & 1)) * W2 + (s & 1);   // fine offset of sub-position s
        bf16x8 af[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt)
            af[nt] = as_bf16x8(*reinterpret_cast<const uint4*>(&wl[(nt * 16 + li) * WS + 8 * g]));
#pragma unroll
        for (int q = 0; q < UPD_VG; ++q) {
            const uint4 gq = vok[q] ? *reinterpret_cast<const uint4*>(gr + (fb[q] + so) * ldg + co0)
                                    : make_uint4(0, 0, 0, 0);
            const bf16x8 gb = as_bf16x8(gq);
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
                acc[q][nt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(af[nt], gb, acc[q][nt], 0, 0, 0);
        }
    }
    // explicit wait states between the last MFMAs and the reads of their
    // results (as in k_up2_mfma)
#pragma unroll
    for (int q = 0; q < UPD_VG; ++q)
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" : "+a"(acc[q][nt]));
#pragma unroll
    for (int q = 0; q < UPD_VG; ++q) {
        if (!vok[q]) continue;
        const int64_t v = vw + 16 * q + li;
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            const int ci = nt * 16 + 4 * g;
            float o[4] = {acc[q][nt][0], acc[q][nt][1], acc[q][nt][2], acc[q][nt][3]};
            if (below) {
                const uint2 m = *reinterpret_cast<const uint2*>(below + v * ldb + ci);
                if (!bf_pos((u16)(m.x & 0xFFFF))) o[0] = 0.0f;
                if (!bf_pos((u16)(m.x >> 16))) o[1] = 0.0f;
                if (!bf_pos((u16)(m.y & 0xFFFF))) o[2] = 0.0f;
                if (!bf_pos((u16)(m.y >> 16))) o[3] = 0.0f;
            }
            uint2 pk;
            pk.x = (uint32_t)f2bf(o[0]) | ((uint32_t)f2bf(o[1]) << 16);
            pk.y = (uint32_t)f2bf(o[2]) | ((uint32_t)f2bf(o[3]) << 16);
            *reinterpret_cast<uint2*>(out + v * ldo + ci) = pk;
        }
    }
}

// weight gradient of up2: dw[co][s][ci] = sum_v g[2v + s][co] x[v][ci].
// Block = (s, co tile of 16, ci tile of 16) x voxel split; thread = one
// (co, ci) output; 64 coarse voxels per LDS round.
__global__ __launch_bounds__(256) void k_up2_wgrad(const u16* __restrict__ x, int ldx, int cin,
                                                   const u16* __restrict__ gr, int ldg, int cout, int n, int d, int h,
                                                   int w, float* __restrict__ partial)
{
    __shared__ float gs[64][17];
    __shared__ float xs_[64][17];
    const int ci_tiles = cin / 16, co_tiles = cout / 16;
    int b = blockIdx.x;
    const int cit = b % ci_tiles;
    b /= ci_tiles;
    const int cot = b % co_tiles;
    const int s = b / co_tiles;
    const int split = blockIdx.y, nsplit = gridDim.y;
    const int tid = threadIdx.x;
    const int co_l = tid >> 4, ci_l = tid & 15;
    const int64_t nvox = (int64_t)n * d * h * w;
    const int64_t nchunks = (nvox + 63) / 64;
    float acc = 0.0f;
    for (int64_t ch = split; ch < nchunks; ch += nsplit) {
        __syncthreads();
        {
            const int vl = tid >> 2, part = tid & 3;  // 64 voxels x 4 groups of 4 channels
            const int64_t v = ch * 64 + vl;
            float fg[4] = {0, 0, 0, 0}, fx[4] = {0, 0, 0, 0};
            if (v < nvox) {
                int64_t r = v;
                const int xx = (int)(r % w);
                r /= w;
                const int yy = (int)(r % h);
                r /= h;
                const int zz = (int)(r % d);
                const int nb = (int)(r / d);
                const int Z = 2 * zz + (s >> 2), Y = 2 * yy + ((s >> 1) & 1), X = 2 * xx + (s & 1);
                const size_t fv = (((size_t)nb * 2 * d + Z) * 2 * h + Y) * 2 * w + X;
                const uint2 qg = *reinterpret_cast<const uint2*>(gr + fv * ldg + cot * 16 + part * 4);
                const uint2 qx = *reinterpret_cast<const uint2*>(x + (size_t)v * ldx + cit * 16 + part * 4);
                fg[0] = __uint_as_float(qg.x << 16); fg[1] = __uint_as_float(qg.x & 0xFFFF0000u);
                fg[2] = __uint_as_float(qg.y << 16); fg[3] = __uint_as_float(qg.y & 0xFFFF0000u);
                fx[0] = __uint_as_float(qx.x << 16); fx[1] = __uint_as_float(qx.x & 0xFFFF0000u);
                fx[2] = __uint_as_float(qx.y << 16); fx[3] = __uint_as_float(qx.y & 0xFFFF0000u);
            }
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                gs[vl][part * 4 + e] = fg[e];
                xs_[vl][part * 4 + e] = fx[e];
            }
        }
        __syncthreads();
#pragma unroll 8
        for (int k = 0; k < 64; ++k) acc = fmaf(gs[k][co_l], xs_[k][ci_l], acc);
    }
    float* part = partial + (size_t)split * cout * 8 * cin;
    part[((size_t)(cot * 16 + co_l) * 8 + s) * cin + cit * 16 + ci_l] = acc;
}

// The same weight gradient on the MFMA: per (s, co tile, ci tile) block a
// 16 x 16 GEMM with K = coarse voxels.  Both operands need 8 consecutive
// voxels per lane, so each wave stages its 64-voxel chunk transposed in
// LDS (g rows as [co][voxel], x rows as [ci][voxel]) and issues two MFMAs;
// the block's four waves take interleaved chunks of its voxel share and add
// their 16 x 16 sums in a fixed order at the end (deterministic partials, the
// same layout as k_up2_wgrad's).
#ifndef CTMI_UP2_WGRAD_MFMA
#define CTMI_UP2_WGRAD_MFMA 1
#endif
constexpr int UPW_S = 72;   // LDS row stride (u16) of a transposed chunk
__global__ __launch_bounds__(256) void k_up2_wgrad_mfma(const u16* __restrict__ x, int ldx, int cin,
                                                        const u16* __restrict__ gr, int ldg, int cout, int n, int d,
                                                        int h, int w, float* __restrict__ partial)
{
    __shared__ __attribute__((aligned(16))) u16 gt[4][16 * UPW_S];
    __shared__ __attribute__((aligned(16))) u16 xt[4][16 * UPW_S];
    __shared__ float red[4][256];
    const int ci_tiles = cin / 16, co_tiles = cout / 16;
    int b = blockIdx.x;
    const int cit = b % ci_tiles;
    b /= ci_tiles;
    const int cot = b % co_tiles;
    const int s = b / co_tiles;
    const int split = blockIdx.y, nsplit = gridDim.y;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, li = lane & 15;
    const int64_t nvox = (int64_t)n * d * h * w;
    const int64_t nchunks = (nvox + 63) / 64;
    const int64_t mine = nchunks > split ? (nchunks - split + nsplit - 1) / nsplit : 0;   // chunks of this split
    const int64_t rounds = (mine + 3) / 4;
    const int D2 = 2 * d, H2 = 2 * h, W2 = 2 * w;
    f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
    for (int64_t it = 0; it < rounds; ++it) {
        const int64_t j = 4 * it + wave;               // this wave's chunk in the split's list
        const int64_t v = (split + j * nsplit) * 64 + lane;
        uint4 g0 = make_uint4(0, 0, 0, 0), g1 = g0, x0 = g0, x1 = g0;
        if (j < mine && v < nvox) {
            int64_t r = v;
            const int cx = (int)(r % w);
            r /= w;
            const int cy = (int)(r % h);
            r /= h;
            const int cz = (int)(r % d);
            const int nb = (int)(r / d);
            const int64_t fv = (((int64_t)nb * D2 + 2 * cz + (s >> 2)) * H2 + 2 * cy + ((s >> 1) & 1)) * W2 + 2 * cx +
                               (s & 1);
            const u16* gp = gr + fv * ldg + cot * 16;
            const u16* xp = x + v * ldx + cit * 16;
            g0 = *reinterpret_cast<const uint4*>(gp);
            g1 = *reinterpret_cast<const uint4*>(gp + 8);
            x0 = *reinterpret_cast<const uint4*>(xp);
            x1 = *reinterpret_cast<const uint4*>(xp + 8);
        }
        __syncthreads();   // every wave has read the previous chunk's fragments
        {
            const uint32_t gw[8] = {g0.x, g0.y, g0.z, g0.w, g1.x, g1.y, g1.z, g1.w};
            const uint32_t xw[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                gt[wave][(2 * c) * UPW_S + lane] = (u16)(gw[c] & 0xFFFFu);
                gt[wave][(2 * c + 1) * UPW_S + lane] = (u16)(gw[c] >> 16);
                xt[wave][(2 * c) * UPW_S + lane] = (u16)(xw[c] & 0xFFFFu);
                xt[wave][(2 * c + 1) * UPW_S + lane] = (u16)(xw[c] >> 16);
            }
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < 64; kk += 32) {
            const uint4 af = *reinterpret_cast<const uint4*>(&gt[wave][li * UPW_S + kk + 8 * g]);
            const uint4 bf = *reinterpret_cast<const uint4*>(&xt[wave][li * UPW_S + kk + 8 * g]);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(af), as_bf16x8(bf), acc, 0, 0, 0);
        }
    }
    asm volatile("s_nop 7\n\ts_nop 7\n\ts_nop 7" : "+a"(acc));
    // lane (li, g) holds dW rows co = 4 g .. 4 g + 3 of column ci = li
#pragma unroll
    for (int e = 0; e < 4; ++e) red[wave][(4 * g + e) * 16 + li] = acc[e];
    __syncthreads();
    const int t = threadIdx.x, co_l = t >> 4, ci_l = t & 15;
    const float sum = ((red[0][t] + red[1][t]) + red[2][t]) + red[3][t];
    float* part = partial + (size_t)split * cout * 8 * cin;
    part[((size_t)(cot * 16 + co_l) * 8 + s) * cin + cit * 16 + ci_l] = sum;
}

// residual head: out[v] = x_in[v] + hb + sum_c hw[c] a[v][c] (FP32)
__global__ void k_head(const float* __restrict__ xin, const u16* __restrict__ act, int lda, int c,
                       const u16* __restrict__ hw, const float* __restrict__ hb, int64_t nvox, float* __restrict__ out)
{
    const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (v >= nvox) return;
    float s = 0.0f;
    for (int c8 = 0; c8 < c; c8 += 8) {
        float fa[8];
        unpack8(*reinterpret_cast<const uint4*>(act + v * lda + c8), fa);
#pragma unroll
        for (int k = 0; k < 8; ++k) s = fmaf(fa[k], bf2f(hw[c8 + k]), s);
    }
    out[v] = xin[v] + (hb[0] + s);
}

// MSE loss through the head (16 channels): g = 2 (out - t) / M; dz[v][c] =
// bf16(g hw[c] mask(a[v][c])); per-block FP64 partial sums of g a[v][c]
// (16 columns), of g, and of (out - t)^2 -> partial[block][18]
constexpr int HEAD_C = 16;

__global__ __launch_bounds__(256) void k_head_loss_bwd(const float* __restrict__ out, const float* __restrict__ tgt,
                                                       const u16* __restrict__ act, int lda,
                                                       const u16* __restrict__ hw, int64_t nvox, double inv_m,
                                                       u16* __restrict__ dz, int ldz, double* __restrict__ partial)
{
    __shared__ double red[256];
    const int tid = threadIdx.x;
    float hwf[HEAD_C];
#pragma unroll
    for (int k = 0; k < HEAD_C; ++k) hwf[k] = bf2f(hw[k]);
    double s[HEAD_C + 2];
#pragma unroll
    for (int k = 0; k < HEAD_C + 2; ++k) s[k] = 0.0;
    for (int64_t v = (int64_t)blockIdx.x * 256 + tid; v < nvox; v += (int64_t)gridDim.x * 256) {
        const float diff = out[v] - tgt[v];
        const float gv = (float)(2.0 * inv_m) * diff;
#pragma unroll
        for (int c8 = 0; c8 < HEAD_C; c8 += 8) {
            float fa[8], o[8];
            unpack8(*reinterpret_cast<const uint4*>(act + v * lda + c8), fa);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                s[c8 + k] += (double)gv * fa[k];
                o[k] = fa[k] > 0.0f ? gv * hwf[c8 + k] : 0.0f;
            }
            *reinterpret_cast<uint4*>(dz + v * ldz + c8) = pack8(o);
        }
        s[HEAD_C] += gv;
        s[HEAD_C + 1] += (double)diff * diff;
    }
#pragma unroll
    for (int k = 0; k < HEAD_C + 2; ++k) {
        red[tid] = s[k];
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st) red[tid] += red[tid + st];
            __syncthreads();
        }
        if (tid == 0) partial[(size_t)blockIdx.x * (HEAD_C + 2) + k] = red[0];
        __syncthreads();
    }
}

// out[i] = sum_s partial[s][i] in FP64 (fixed order); the first nf sums
// also go to outf as FP32 when outf is given
__global__ void k_sum_partials64(const double* __restrict__ partial, int nsplit, int n, double* __restrict__ out,
                                 float* __restrict__ outf, int nf)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int k = 0; k < nsplit; ++k) s += partial[(size_t)k * n + i];
    out[i] = s;
    if (outf && i < nf) outf[i] = (float)s;
}

// Adam on FP32 master weights (bias-corrected step sizes from the host):
// m = b1 m + (1 - b1) g; v = b2 v + (1 - b2) g^2;
// w -= lr_t m / (sqrt(v) / sqrt(1 - b2^t) + eps), lr_t = lr / (1 - b1^t)
__global__ void k_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                       const float* __restrict__ gr, int64_t n, float b1, float b2, float lr_t, float inv_sqrt_bc2,
                       float eps)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float g = gr[i];
    const float mi = fmaf(b1, m[i], (1.0f - b1) * g);
    const float vi = fmaf(b2, v[i], (1.0f - b2) * g * g);
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr_t * mi / (sqrtf(vi) * inv_sqrt_bc2 + eps);
}

// FP32 [cout][27][cin] -> BF16 forward weights (same layout) and, if wd is
// given, BF16 data-gradient weights wd[ci][26 - t][co]
__global__ void k_pack_conv3(const float* __restrict__ w, int cout, int cin, u16* __restrict__ wf, u16* __restrict__ wd)
{
    const int64_t n = (int64_t)cout * 27 * cin;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int ci = (int)(i % cin);
    const int t = (int)((i / cin) % 27);
    const int co = (int)(i / ((int64_t)27 * cin));
    const u16 q = f2bf(w[i]);
    wf[i] = q;
    if (wd) wd[((size_t)ci * 27 + (26 - t)) * cout + co] = q;
}

__global__ void k_to_bf16(const float* __restrict__ a, int64_t n, u16* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = f2bf(a[i]);
}

inline unsigned blocks_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_unet_conv3(const UnetConv3& a, hipStream_t s)
{
    const int tiles_x = (a.w + CX - 1) / CX, tiles_y = (a.h + CY - 1) / CY, tiles_z = (a.d + CZ - 1) / CZ;
    dim3 grid(tiles_x * tiles_y, tiles_z, a.n);
    switch (a.cout) {
    case 16: k_conv3<1><<<grid, 256, 0, s>>>(a); break;
    case 32: k_conv3<2><<<grid, 256, 0, s>>>(a); break;
    case 64: k_conv3<4><<<grid, 256, 0, s>>>(a); break;
    case 128: k_conv3<8><<<grid, 256, 0, s>>>(a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

int unet_wgrad_splits(int n, int d, int h, int w, int cin, int cout)
{
    const int64_t tiles = (int64_t)n * ((d + CZ - 1) / CZ) * ((h + CY - 1) / CY) * ((w + CX - 1) / CX);
    const int pairs = (cin / 16) * (cout / 16);
    int64_t sp = 1024 / pairs;
    if (sp < 1) sp = 1;
    if (sp > tiles) sp = tiles;
    return (int)sp;
}

size_t unet_wgrad_ws_bytes(int n, int d, int h, int w, int cin, int cout)
{
    const size_t a = (size_t)unet_wgrad_splits(n, d, h, w, cin, cout) * cout * 27 * cin * sizeof(float);
    const size_t b = (size_t)1024 * cout * sizeof(float);  // channel-sum partials
    return a > b ? a : b;
}

hipError_t launch_unet_conv3_wgrad(const UnetWgrad& a, float* dw, float* db, int accumulate, hipStream_t s)
{
    const int cin = a.c0 + a.c1;
    const int nsplit = unet_wgrad_splits(a.n, a.d, a.h, a.w, cin, a.cout);
    dim3 grid((cin / 16) * (a.cout / 16), nsplit);
    k_conv3_wgrad<<<grid, 256, 0, s>>>(a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nw = (int64_t)a.cout * 27 * cin;
    k_sum_partials<<<blocks_for(nw, SUM_E), 256, 0, s>>>(a.partial, nsplit, nw, dw, accumulate);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (db) {
        const int64_t nvox = (int64_t)a.n * a.d * a.h * a.w;
        int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, nvox / 1024));
        k_channel_sums<<<nb, 256, 0, s>>>(a.dz, a.ldz, a.cout, nvox, a.partial);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_sum_partials<<<blocks_for(a.cout, SUM_E), 256, 0, s>>>(a.partial, nb, a.cout, db, accumulate);
    }
    return hipGetLastError();
}

hipError_t launch_unet_pack_input(const float* x, int64_t nvox, uint16_t* out, hipStream_t s)
{
    k_pack_input<<<blocks_for(nvox, 256), 256, 0, s>>>(x, nvox, out);
    return hipGetLastError();
}

hipError_t launch_unet_pool2(const uint16_t* in, int ldi, int n, int d, int h, int w, int c, uint16_t* out, int ldo,
                             hipStream_t s)
{
    const int64_t total = (int64_t)n * d * h * w * (c / 8);
    k_pool2<<<blocks_for(total, 256), 256, 0, s>>>(in, ldi, n, d, h, w, c, out, ldo);
    return hipGetLastError();
}

hipError_t launch_unet_skip_grad(const uint16_t* e, int lde, const uint16_t* dp, int ldp, const uint16_t* dcat,
                                 int ldc, int n, int d, int h, int w, int c, uint16_t* out, int ldo, hipStream_t s)
{
    const int64_t total = (int64_t)n * d * h * w * (c / 8);
    k_skip_grad<<<blocks_for(total, 256), 256, 0, s>>>(e, lde, dp, ldp, dcat, ldc, n, d, h, w, c, out, ldo);
    return hipGetLastError();
}

hipError_t launch_unet_up2(const uint16_t* x, int ldx, int cin, const uint16_t* wt, const float* bias, int cout,
                           int n, int d, int h, int w, uint16_t* out, int ldo, hipStream_t s)
{
    const int64_t nvox = (int64_t)n * d * h * w;
    if (cin % 32 == 0 && (cout == 16 || cout == 32 || cout == 64)) {
        // one wave per 16 coarse voxels, four waves per workgroup
        const unsigned blocks = (unsigned)((nvox + 63) / 64);
        if (cout == 16)
            k_up2_mfma<1><<<blocks, 256, 0, s>>>(x, ldx, cin, wt, bias, n, d, h, w, out, ldo);
        else if (cout == 32)
            k_up2_mfma<2><<<blocks, 256, 0, s>>>(x, ldx, cin, wt, bias, n, d, h, w, out, ldo);
        else
            k_up2_mfma<4><<<blocks, 256, 0, s>>>(x, ldx, cin, wt, bias, n, d, h, w, out, ldo);
        return hipGetLastError();
    }
    const int64_t total = nvox * 8 * (cout / 8);
    k_up2<<<blocks_for(total, 256), 256, 0, s>>>(x, ldx, cin, wt, bias, cout, n, d, h, w, out, ldo);
    return hipGetLastError();
}

hipError_t launch_unet_up2_dgrad(const uint16_t* g, int ldg, int cout, const uint16_t* wt, int cin,
                                 const uint16_t* below, int ldb, int n, int d, int h, int w, uint16_t* out, int ldo,
                                 hipStream_t s)
{
    const int64_t nvox = (int64_t)n * d * h * w;
    if (CTMI_UP2_DGRAD_MFMA && cout % 16 == 0 && (cin == 32 || cin == 64 || cin == 128)) {
        const unsigned blocks = (unsigned)((nvox + 4 * 16 * UPD_VG - 1) / (4 * 16 * UPD_VG));
        if (cin == 32) k_up2_dgrad_mfma<2><<<blocks, 256, 0, s>>>(g, ldg, cout, wt, below, ldb, n, d, h, w, out, ldo);
        else if (cin == 64) k_up2_dgrad_mfma<4><<<blocks, 256, 0, s>>>(g, ldg, cout, wt, below, ldb, n, d, h, w, out, ldo);
        else k_up2_dgrad_mfma<8><<<blocks, 256, 0, s>>>(g, ldg, cout, wt, below, ldb, n, d, h, w, out, ldo);
        return hipGetLastError();
    }
    const int64_t total = nvox * (cin / 8);
    k_up2_dgrad<<<blocks_for(total, 256), 256, 0, s>>>(g, ldg, cout, wt, cin, below, ldb, n, d, h, w, out, ldo);
    return hipGetLastError();
}

int unet_up2_wgrad_splits(int n, int d, int h, int w, int cin, int cout)
{
    const int64_t chunks = ((int64_t)n * d * h * w + 63) / 64;
    const int blocks = 8 * (cin / 16) * (cout / 16);
    int64_t sp = 2048 / blocks;
    if (sp < 1) sp = 1;
    if (sp > chunks) sp = chunks;
    return (int)sp;
}

size_t unet_up2_wgrad_ws_bytes(int n, int d, int h, int w, int cin, int cout)
{
    const size_t a = (size_t)unet_up2_wgrad_splits(n, d, h, w, cin, cout) * cout * 8 * cin * sizeof(float);
    const size_t b = (size_t)1024 * cout * sizeof(float);
    return a > b ? a : b;
}

hipError_t launch_unet_up2_wgrad(const uint16_t* x, int ldx, int cin, const uint16_t* g, int ldg, int cout, int n,
                                 int d, int h, int w, float* ws, float* dw, float* db, int accumulate, hipStream_t s)
{
    const int nsplit = unet_up2_wgrad_splits(n, d, h, w, cin, cout);
    dim3 grid(8 * (cin / 16) * (cout / 16), nsplit);
    if (CTMI_UP2_WGRAD_MFMA)
        k_up2_wgrad_mfma<<<grid, 256, 0, s>>>(x, ldx, cin, g, ldg, cout, n, d, h, w, ws);
    else
        k_up2_wgrad<<<grid, 256, 0, s>>>(x, ldx, cin, g, ldg, cout, n, d, h, w, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nw = (int64_t)cout * 8 * cin;
    k_sum_partials<<<blocks_for(nw, SUM_E), 256, 0, s>>>(ws, nsplit, nw, dw, accumulate);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (db) {
        const int64_t nvox = (int64_t)n * 8 * d * h * w;
        int nb = (int)std::min<int64_t>(1024, std::max<int64_t>(1, nvox / 1024));
        k_channel_sums<<<nb, 256, 0, s>>>(g, ldg, cout, nvox, ws);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        k_sum_partials<<<blocks_for(cout, SUM_E), 256, 0, s>>>(ws, nb, cout, db, accumulate);
    }
    return hipGetLastError();
}

hipError_t launch_unet_head(const float* xin, const uint16_t* act, int lda, int c, const uint16_t* hw,
                            const float* hb, int64_t nvox, float* out, hipStream_t s)
{
    k_head<<<blocks_for(nvox, 256), 256, 0, s>>>(xin, act, lda, c, hw, hb, nvox, out);
    return hipGetLastError();
}

size_t unet_head_ws_bytes() { return (size_t)512 * (HEAD_C + 2) * sizeof(double); }

hipError_t launch_unet_head_loss_bwd(const float* out, const float* tgt, const uint16_t* act, int lda,
                                     const uint16_t* hw, int64_t nvox, uint16_t* dz, int ldz, double* ws,
                                     double* sums, float* dhead, hipStream_t s)
{
    const int nb = (int)std::min<int64_t>(512, std::max<int64_t>(1, (nvox + 255) / 256));
    k_head_loss_bwd<<<nb, 256, 0, s>>>(out, tgt, act, lda, hw, nvox, 1.0 / (double)nvox, dz, ldz, ws);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    k_sum_partials64<<<1, 64, 0, s>>>(ws, nb, HEAD_C + 2, sums, dhead, HEAD_C + 1);
    return hipGetLastError();
}

hipError_t launch_unet_adam(float* w, float* m, float* v, const float* g, int64_t n, float b1, float b2, float lr_t,
                            float inv_sqrt_bc2, float eps, hipStream_t s)
{
    k_adam<<<blocks_for(n, 256), 256, 0, s>>>(w, m, v, g, n, b1, b2, lr_t, inv_sqrt_bc2, eps);
    return hipGetLastError();
}

hipError_t launch_unet_pack_conv3(const float* w, int cout, int cin, uint16_t* wf, uint16_t* wd, hipStream_t s)
{
    k_pack_conv3<<<blocks_for((int64_t)cout * 27 * cin, 256), 256, 0, s>>>(w, cout, cin, wf, wd);
    return hipGetLastError();
}

hipError_t launch_unet_to_bf16(const float* a, int64_t n, uint16_t* out, hipStream_t s)
{
    k_to_bf16<<<blocks_for(n, 256), 256, 0, s>>>(a, n, out);
    return hipGetLastError();
}

}  // namespace ctmi
