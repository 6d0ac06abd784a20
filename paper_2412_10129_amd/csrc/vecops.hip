// Vector kernels of the iterative methods: CGLS (section 2.2.1), OS-SART
// (section 2.2.2) and the error history (section 2.2.3).  All are streaming
// HBM-bound loops; reductions accumulate in FP64 with a fixed blocking and
// a fixed tree order, so results are bit-reproducible for a given n.
#include "ctmi_internal.h"

namespace ctmi {

namespace {

constexpr int RB = 256;          // threads per reduction block
constexpr int RMAX = 1024;       // max partial sums

__device__ __forceinline__ double block_sum(double v, double* sh)
{
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = RB / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    return sh[0];
}

__global__ void __launch_bounds__(RB) k_final_sum(const double* __restrict__ part, int nparts, int nvals,
                                                  double* out)
{
    __shared__ double sh[RB];
    for (int c = 0; c < nvals; ++c) {
        double s = 0.0;
        for (int i = threadIdx.x; i < nparts; i += RB) s += part[c * RMAX + i];
        s = block_sum(s, sh);
        if (threadIdx.x == 0) out[c] = s;
        __syncthreads();
    }
}

// Partial FP64 dot products, one per block (a fixed blocking: the result
// depends only on n).  With V4 (both arrays 16-byte aligned) each lane
// takes float4 pairs, two per step so that four loads are in flight; block
// 0 adds the n mod 4 tail.  Products of two floats are exact in FP64.
template <bool V4>
__global__ void __launch_bounds__(RB) k_dot_partial(const float* __restrict__ a, const float* __restrict__ b,
                                                    int64_t n, double* __restrict__ part)
{
    __shared__ double sh[RB];
    double s = 0.0, t = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RB;
    if (V4) {
        const float4* __restrict__ a4 = reinterpret_cast<const float4*>(a);
        const float4* __restrict__ b4 = reinterpret_cast<const float4*>(b);
        const int64_t n4 = n >> 2;
        int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
        for (; i + stride < n4; i += 2 * stride) {
            const float4 x0 = a4[i], y0 = b4[i], x1 = a4[i + stride], y1 = b4[i + stride];
            s = __builtin_fma((double)x0.x, (double)y0.x, s);
            t = __builtin_fma((double)x1.x, (double)y1.x, t);
            s = __builtin_fma((double)x0.y, (double)y0.y, s);
            t = __builtin_fma((double)x1.y, (double)y1.y, t);
            s = __builtin_fma((double)x0.z, (double)y0.z, s);
            t = __builtin_fma((double)x1.z, (double)y1.z, t);
            s = __builtin_fma((double)x0.w, (double)y0.w, s);
            t = __builtin_fma((double)x1.w, (double)y1.w, t);
        }
        if (i < n4) {
            const float4 x0 = a4[i], y0 = b4[i];
            s = __builtin_fma((double)x0.x, (double)y0.x, s);
            s = __builtin_fma((double)x0.y, (double)y0.y, s);
            s = __builtin_fma((double)x0.z, (double)y0.z, s);
            s = __builtin_fma((double)x0.w, (double)y0.w, s);
        }
        if (blockIdx.x == 0 && (int64_t)threadIdx.x < (n & 3)) {
            const int64_t k = 4 * n4 + threadIdx.x;
            t = __builtin_fma((double)a[k], (double)b[k], t);
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += stride)
            s += (double)a[i] * (double)b[i];
    }
    s = block_sum(s + t, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_axpby(int64_t n, float a, const float* __restrict__ x, float b,
                                               float* __restrict__ y)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        y[i] = __builtin_fmaf(a, x[i], b * y[i]);
}

__device__ __forceinline__ float safe_ratio(const double* num, const double* den)
{
    const double d = *den;
    return d != 0.0 ? (float)(*num / d) : 0.0f;
}

__global__ void __launch_bounds__(256) k_cgls_x(float* __restrict__ x, const float* __restrict__ p, int64_t n,
                                                const double* gamma, const double* delta)
{
    const float alpha = safe_ratio(gamma, delta);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] = __builtin_fmaf(alpha, p[i], x[i]);
}

// r -= alpha q with |r|^2 (FP64) per block; V4 as in k_dot_partial.
template <bool V4>
__global__ void __launch_bounds__(RB) k_cgls_r(float* __restrict__ r, const float* __restrict__ q, int64_t n,
                                               const double* gamma, const double* delta, double* __restrict__ part)
{
    __shared__ double sh[RB];
    const float alpha = safe_ratio(gamma, delta);
    double s = 0.0, t = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RB;
    if (V4) {
        float4* __restrict__ r4 = reinterpret_cast<float4*>(r);
        const float4* __restrict__ q4 = reinterpret_cast<const float4*>(q);
        const int64_t n4 = n >> 2;
        int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x;
        for (; i + stride < n4; i += 2 * stride) {
            float4 x0 = r4[i], x1 = r4[i + stride];
            const float4 y0 = q4[i], y1 = q4[i + stride];
            x0.x = __builtin_fmaf(-alpha, y0.x, x0.x);
            x0.y = __builtin_fmaf(-alpha, y0.y, x0.y);
            x0.z = __builtin_fmaf(-alpha, y0.z, x0.z);
            x0.w = __builtin_fmaf(-alpha, y0.w, x0.w);
            x1.x = __builtin_fmaf(-alpha, y1.x, x1.x);
            x1.y = __builtin_fmaf(-alpha, y1.y, x1.y);
            x1.z = __builtin_fmaf(-alpha, y1.z, x1.z);
            x1.w = __builtin_fmaf(-alpha, y1.w, x1.w);
            r4[i] = x0;
            r4[i + stride] = x1;
            s = __builtin_fma((double)x0.x, (double)x0.x, s);
            t = __builtin_fma((double)x1.x, (double)x1.x, t);
            s = __builtin_fma((double)x0.y, (double)x0.y, s);
            t = __builtin_fma((double)x1.y, (double)x1.y, t);
            s = __builtin_fma((double)x0.z, (double)x0.z, s);
            t = __builtin_fma((double)x1.z, (double)x1.z, t);
            s = __builtin_fma((double)x0.w, (double)x0.w, s);
            t = __builtin_fma((double)x1.w, (double)x1.w, t);
        }
        if (i < n4) {
            float4 x0 = r4[i];
            const float4 y0 = q4[i];
            x0.x = __builtin_fmaf(-alpha, y0.x, x0.x);
            x0.y = __builtin_fmaf(-alpha, y0.y, x0.y);
            x0.z = __builtin_fmaf(-alpha, y0.z, x0.z);
            x0.w = __builtin_fmaf(-alpha, y0.w, x0.w);
            r4[i] = x0;
            s = __builtin_fma((double)x0.x, (double)x0.x, s);
            s = __builtin_fma((double)x0.y, (double)x0.y, s);
            s = __builtin_fma((double)x0.z, (double)x0.z, s);
            s = __builtin_fma((double)x0.w, (double)x0.w, s);
        }
        if (blockIdx.x == 0 && (int64_t)threadIdx.x < (n & 3)) {
            const int64_t k = 4 * n4 + threadIdx.x;
            const float v = __builtin_fmaf(-alpha, q[k], r[k]);
            r[k] = v;
            t = __builtin_fma((double)v, (double)v, t);
        }
    } else {
        for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += stride) {
            const float v = __builtin_fmaf(-alpha, q[i], r[i]);
            r[i] = v;
            s += (double)v * (double)v;
        }
    }
    s = block_sum(s + t, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_cgls_p(float* __restrict__ p, const float* __restrict__ s_, int64_t n,
                                                const double* g0, const double* g1)
{
    const float beta = safe_ratio(g1, g0);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        p[i] = __builtin_fmaf(beta, p[i], s_[i]);
}

__global__ void __launch_bounds__(256) k_recip(const float* in, float* out, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float v = in[i];
        out[i] = v != 0.0f ? 1.0f / v : 0.0f;
    }
}

__global__ void __launch_bounds__(256) k_sart_residual(const float* __restrict__ b, const float* ax,
                                                       const float* __restrict__ w, float* out, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        out[i] = w[i] * (b[i] - ax[i]);
}

__global__ void __launch_bounds__(256) k_sart_update(float* __restrict__ x, const float* __restrict__ v,
                                                     const float* __restrict__ bp, int64_t n, float lam, int nonneg)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float y = __builtin_fmaf(lam * v[i], bp[i], x[i]);
        if (nonneg) y = fmaxf(y, 0.0f);
        x[i] = y;
    }
}

// Adaptive-weighted TV (section 2.2.3, extended to 3-D): the term of voxel
// u (all three backward neighbours present) is s_u = sqrt(sum_a w_a d_a^2 +
// eps), d_a = x_u - x_{u - e_a}, w_a = exp(-(d_a / delta)^2) (1 for plain
// TV); q_a(u) = w_a d_a / s_u (0 when s_u = 0).  The gradient with the
// weights lagged is g_v = sum_a q_a(v) - sum_a q_a(v + e_a).  One thread per
// voxel reads its 13-point neighbourhood (neighbouring threads share it
// through the caches) and forms the four terms it needs.
struct TvTerm {
    float qz, qy, qx;
};

__device__ __forceinline__ TvTerm tv_term(float c, float bz, float by, float bx, float nid2, float eps)
{
    const float dz = c - bz, dy = c - by, dx = c - bx;
    float wz = 1.0f, wy = 1.0f, wx = 1.0f;
    if (nid2 != 0.0f) {   // nid2 = -1 / delta^2
        wz = __expf(dz * dz * nid2);
        wy = __expf(dy * dy * nid2);
        wx = __expf(dx * dx * nid2);
    }
    const float az = wz * dz, ay = wy * dy, ax = wx * dx;
    const float s2 = __builtin_fmaf(az, dz, __builtin_fmaf(ay, dy, __builtin_fmaf(ax, dx, eps)));
    const float r = s2 > 0.0f ? 1.0f / __builtin_sqrtf(s2) : 0.0f;
    return TvTerm{az * r, ay * r, ax * r};
}

// Tiled form: a workgroup owns a 64 x 8 (x, y) column of the volume over
// TZ consecutive planes and marches up z.  Each step stages plane z + 1 (with
// a one-voxel lower halo in x and y) in LDS, forms the terms of plane z + 1
// once for the tile and its upper halo, and finishes plane z's gradient from
// the terms of planes z and z + 1.  The plane after is loaded into registers
// while the step runs.
constexpr int TVX = 64, TVY = 8, TVZ = 64;
constexpr int TXH = TVX + 2, TYH = TVY + 2;          // staged plane with lower and upper halo
constexpr int TQX = TVX + 1, TQY = TVY + 1;          // terms: tile plus upper halo
constexpr int TVL = (TXH * TYH + 255) / 256;         // staged cells per thread

__global__ void __launch_bounds__(256) k_awtv_grad(const float* __restrict__ x, float* __restrict__ g, int nz, int ny,
                                                   int nx, float nid2, float eps)
{
    __shared__ float pl[2][TXH * TYH];   // planes z and z + 1 (x from x0 - 1, y from y0 - 1)
    __shared__ float q[2][3][TQX * TQY]; // terms (z, y, x components) of planes z and z + 1
    const int tid = threadIdx.x;
    const int x0 = blockIdx.x * TVX, y0 = blockIdx.y * TVY, z0 = blockIdx.z * TVZ;
    const int z1 = min(z0 + TVZ, nz);
    const int64_t sz = (int64_t)nx * ny;
    // staged cells of this thread: c -> (x0 - 1 + c % TXH, y0 - 1 + c / TXH)
    int64_t off[TVL];
    bool in[TVL];
#pragma unroll
    for (int m = 0; m < TVL; ++m) {
        const int c = tid + 256 * m;
        const int X = x0 - 1 + c % TXH, Y = y0 - 1 + c / TXH;
        in[m] = c < TXH * TYH && X >= 0 && X < nx && Y >= 0 && Y < ny;
        off[m] = in[m] ? (int64_t)Y * nx + X : 0;
    }
    auto fetch = [&](int Z, float (&r)[TVL]) {
#pragma unroll
        for (int m = 0; m < TVL; ++m) r[m] = (in[m] && Z >= 0 && Z < nz) ? x[(int64_t)Z * sz + off[m]] : 0.0f;
    };
    auto stage = [&](float* dst, const float (&r)[TVL]) {
#pragma unroll
        for (int m = 0; m < TVL; ++m) {
            const int c = tid + 256 * m;
            if (c < TXH * TYH) dst[c] = r[m];
        }
    };
    // terms of plane Z from its staged plane cur and the plane below, prev
    auto terms = [&](int Z, const float* cur, const float* prev, int slot) {
        for (int c = tid; c < TQX * TQY; c += 256) {
            const int i = c % TQX, j = c / TQX;
            const int X = x0 + i, Y = y0 + j;
            float qz = 0.0f, qy = 0.0f, qx = 0.0f;
            if (X >= 1 && Y >= 1 && Z >= 1 && X < nx && Y < ny && Z < nz) {
                const int k = (j + 1) * TXH + (i + 1);
                const TvTerm t = tv_term(cur[k], prev[k], cur[k - TXH], cur[k - 1], nid2, eps);
                qz = t.qz;
                qy = t.qy;
                qx = t.qx;
            }
            q[slot][0][c] = qz;
            q[slot][1][c] = qy;
            q[slot][2][c] = qx;
        }
    };
    int cp = 0, cq = 0;   // LDS slots holding plane z and its terms
    {
        float r[TVL];
        fetch(z0 - 1, r);
        stage(pl[1], r);
        fetch(z0, r);
        stage(pl[0], r);
    }
    __syncthreads();
    terms(z0, pl[0], pl[1], 0);
    // planes z + 1 ... z + 4 in flight in registers (global-load latency is
    // longer than one step)
    float ra[TVL], rb[TVL], rc[TVL], rd[TVL];
    fetch(z0 + 1, ra);
    fetch(z0 + 2, rb);
    fetch(z0 + 3, rc);
    fetch(z0 + 4, rd);
    auto step = [&](int z, float (&r)[TVL]) {
        // stage plane z + 1 over the slot of plane z - 1, then refill the
        // registers with plane z + 5
        stage(pl[cp ^ 1], r);
        __syncthreads();
        fetch(z + 5, r);
        terms(z + 1, pl[cp ^ 1], pl[cp], cq ^ 1);
        __syncthreads();
#pragma unroll
        for (int o = tid; o < TVX * TVY; o += 256) {
            const int tx = o % TVX, ty = o / TVX;
            const int X = x0 + tx, Y = y0 + ty;
            if (X < nx && Y < ny) {
                const int k = ty * TQX + tx;
                const float gv = q[cq][0][k] + q[cq][1][k] + q[cq][2][k] - q[cq ^ 1][0][k] - q[cq][1][k + TQX] -
                                 q[cq][2][k + 1];
                g[(int64_t)z * sz + (int64_t)Y * nx + X] = gv;
            }
        }
        cp ^= 1;
        cq ^= 1;
    };
    for (int z = z0; z < z1; z += 4) {
        step(z, ra);
        if (z + 1 < z1) step(z + 1, rb);
        if (z + 2 < z1) step(z + 2, rc);
        if (z + 3 < z1) step(z + 3, rd);
    }
}

// TV steepest-descent step: x -= step * g / sqrt(gnorm2) (gnorm2 a device
// double; nothing happens when it is 0).
__global__ void __launch_bounds__(256) k_tv_step(float* __restrict__ x, const float* __restrict__ g, int64_t n,
                                                 const double* __restrict__ gnorm2, float step)
{
    const double gn2 = *gnorm2;
    if (!(gn2 > 0.0)) return;
    const float f = (float)((double)step / sqrt(gn2));
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        x[i] = __builtin_fmaf(-f, g[i], x[i]);
}

// EM ratio (MLEM/OSEM, section 2.2): out = b / ax where ax > 0, else 0.
__global__ void __launch_bounds__(256) k_em_ratio(const float* __restrict__ b, const float* ax, float* out, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const float a = ax[i];
        out[i] = a > 0.0f ? b[i] / a : 0.0f;
    }
}

// EM update: x = x * v * bp, v = 1 / (A^T 1) (0 where no ray reaches).
__global__ void __launch_bounds__(256) k_em_update(float* __restrict__ x, const float* __restrict__ v,
                                                   const float* __restrict__ bp, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) x[i] = x[i] * v[i] * bp[i];
}

__global__ void __launch_bounds__(RB) k_fov_partial(const float* __restrict__ x, const float* __restrict__ gt,
                                                    VolDims v, float cx, float cy, float r2,
                                                    double* __restrict__ part)
{
    __shared__ double sh[RB];
    const int64_t n = (int64_t)v.nx * v.ny * v.nz;
    double s = 0.0, c = 0.0;
    const int64_t stride = (int64_t)gridDim.x * RB;
    for (int64_t i = (int64_t)blockIdx.x * RB + threadIdx.x; i < n; i += stride) {
        const int ix = (int)(i % v.nx);
        const int iy = (int)((i / v.nx) % v.ny);
        const float X = ((float)ix - cx) * v.hx, Y = ((float)iy - cy) * v.hy;
        if (__builtin_fmaf(X, X, Y * Y) <= r2) {
            const double d = (double)x[i] - (double)gt[i];
            s += d * d;
            c += 1.0;
        }
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) part[blockIdx.x] = s;
    __syncthreads();
    c = block_sum(c, sh);
    if (threadIdx.x == 0) part[RMAX + blockIdx.x] = c;
}

unsigned stream_blocks(int64_t n)
{
    int64_t b = (n + 256 * 8 - 1) / (256 * 8);
    if (b < 1) b = 1;
    if (b > 8192) b = 8192;
    return (unsigned)b;
}

}  // namespace

static bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

int reduce_blocks(int64_t n)
{
    int64_t b = (n + RB * 16 - 1) / (RB * 16);
    if (b < 1) b = 1;
    if (b > RMAX) b = RMAX;
    return (int)b;
}

hipError_t launch_dot(const float* a, const float* b, int64_t n, double* out, double* ws, hipStream_t s)
{
    const int g = reduce_blocks(n);
    if (aligned16(a) && aligned16(b))
        hipLaunchKernelGGL(k_dot_partial<true>, dim3(g), dim3(RB), 0, s, a, b, n, ws);
    else
        hipLaunchKernelGGL(k_dot_partial<false>, dim3(g), dim3(RB), 0, s, a, b, n, ws);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(RB), 0, s, ws, g, 1, out);
    return hipGetLastError();
}

hipError_t launch_axpby(int64_t n, float a, const float* x, float b, float* y, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpby, dim3(stream_blocks(n)), dim3(256), 0, s, n, a, x, b, y);
    return hipGetLastError();
}

hipError_t launch_cgls_xr(float* x, const float* p, int64_t nvol, float* r, const float* q, int64_t nproj,
                          const double* gamma, const double* delta, double* rnorm2, double* ws, hipStream_t s)
{
    hipLaunchKernelGGL(k_cgls_x, dim3(stream_blocks(nvol)), dim3(256), 0, s, x, p, nvol, gamma, delta);
    const int g = reduce_blocks(nproj);
    if (aligned16(r) && aligned16(q))
        hipLaunchKernelGGL(k_cgls_r<true>, dim3(g), dim3(RB), 0, s, r, q, nproj, gamma, delta, ws);
    else
        hipLaunchKernelGGL(k_cgls_r<false>, dim3(g), dim3(RB), 0, s, r, q, nproj, gamma, delta, ws);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(RB), 0, s, ws, g, 1, rnorm2);
    return hipGetLastError();
}

hipError_t launch_cgls_p(float* p, const float* s_, int64_t n, const double* g0, const double* g1, hipStream_t s)
{
    hipLaunchKernelGGL(k_cgls_p, dim3(stream_blocks(n)), dim3(256), 0, s, p, s_, n, g0, g1);
    return hipGetLastError();
}

hipError_t launch_recip(const float* in, float* out, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_recip, dim3(stream_blocks(n)), dim3(256), 0, s, in, out, n);
    return hipGetLastError();
}

hipError_t launch_sart_residual(const float* b, const float* ax, const float* w, float* out, int64_t n,
                                hipStream_t s)
{
    hipLaunchKernelGGL(k_sart_residual, dim3(stream_blocks(n)), dim3(256), 0, s, b, ax, w, out, n);
    return hipGetLastError();
}

hipError_t launch_sart_update(float* x, const float* v, const float* bp, int64_t n, float lam, int nonneg,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_sart_update, dim3(stream_blocks(n)), dim3(256), 0, s, x, v, bp, n, lam, nonneg);
    return hipGetLastError();
}

hipError_t launch_awtv_grad(const float* x, float* g, int nz, int ny, int nx, float delta, float eps, hipStream_t s)
{
    // -1 / delta^2, or 0 for plain TV (delta <= 0 or infinite)
    const float nid2 = (delta > 0.0f && delta < CTMI_INF) ? -1.0f / (delta * delta) : 0.0f;
    const dim3 grid((unsigned)((nx + TVX - 1) / TVX), (unsigned)((ny + TVY - 1) / TVY), (unsigned)((nz + TVZ - 1) / TVZ));
    hipLaunchKernelGGL(k_awtv_grad, grid, dim3(256), 0, s, x, g, nz, ny, nx, nid2, eps);
    return hipGetLastError();
}

hipError_t launch_tv_step(float* x, const float* g, int64_t n, const double* gnorm2, float step, hipStream_t s)
{
    hipLaunchKernelGGL(k_tv_step, dim3(stream_blocks(n)), dim3(256), 0, s, x, g, n, gnorm2, step);
    return hipGetLastError();
}

hipError_t launch_em_ratio(const float* b, const float* ax, float* out, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_em_ratio, dim3(stream_blocks(n)), dim3(256), 0, s, b, ax, out, n);
    return hipGetLastError();
}

hipError_t launch_em_update(float* x, const float* v, const float* bp, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_em_update, dim3(stream_blocks(n)), dim3(256), 0, s, x, v, bp, n);
    return hipGetLastError();
}

hipError_t launch_fov_sq_err(const Plan& p, const float* x, const float* gt, double* out, double* ws,
                             hipStream_t s)
{
    const int64_t n = (int64_t)p.vol.nx * p.vol.ny * p.vol.nz;
    const int g = reduce_blocks(n);
    // voxel-centre index of the volume centre; the cylinder is centred on the
    // volume (its offset does not change the index geometry)
    const float cx = 0.5f * (float)p.vol.nx - 0.5f, cy = 0.5f * (float)p.vol.ny - 0.5f;
    const double R = 0.5 * ((double)p.vol.ny * p.vol.hy < (double)p.vol.nx * p.vol.hx ? (double)p.vol.ny * p.vol.hy
                                                                                       : (double)p.vol.nx * p.vol.hx);
    hipLaunchKernelGGL(k_fov_partial, dim3(g), dim3(RB), 0, s, x, gt, p.vol, cx, cy, (float)(R * R), ws);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(RB), 0, s, ws, g, 2, out);
    return hipGetLastError();
}

size_t reduce_ws_bytes() { return sizeof(double) * 2 * RMAX; }

}  // namespace ctmi
