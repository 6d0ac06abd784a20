// FDK (section 2.1, direct methods; Feldkamp-Davis-Kress 1984): the row
// filter (cosine weight, optional Wang offset-detector weight, Ram-Lak ramp
// as a zero-padded FFT convolution, angular scale) and the voxel-driven
// backprojector sum_views (DSO/U)^2 bilinear(q; u, v).
#include "ctmi_internal.h"

namespace ctmi {

namespace {

// ------------------------------------------------------------ backprojector
// One thread per (x, y) voxel column segment of ZC voxels; every view of the
// call is accumulated in registers, so each output voxel is written once.
// On a circular orbit W and fu do not depend on z, so per view a thread
// computes one reciprocal and then walks its ZC voxels along v.
constexpr int FDK_TX = 32, FDK_TY = 8, FDK_ZC = 8;
#ifndef CTMI_FDK_XCD
#define CTMI_FDK_XCD 0
#endif

__global__ void __launch_bounds__(FDK_TX* FDK_TY) k_backward_fdk(const float* __restrict__ proj,
                                                                 float* __restrict__ vol,
                                                                 const ViewGeo* __restrict__ tab, int view0,
                                                                 int nviews, VolDims v, DetDims det, int nbx,
                                                                 int nby, float beta)
{
    const int b = CTMI_FDK_XCD ? (int)xcd_contiguous(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int ix = bx * FDK_TX + (int)(threadIdx.x % FDK_TX);
    const int iy = by * FDK_TY + (int)(threadIdx.x / FDK_TX);
    const int iz0 = bz * FDK_ZC;
    if (ix >= v.nx || iy >= v.ny) return;
    const float fx = (float)ix, fy = (float)iy, fz0 = (float)iz0;
    float acc[FDK_ZC];
#pragma unroll
    for (int z = 0; z < FDK_ZC; ++z) acc[z] = 0.0f;

    for (int k = 0; k < nviews; ++k) {
        const ViewGeo& g = tab[view0 + k];
        const float W = __builtin_fmaf(g.MW[0], fx, __builtin_fmaf(g.MW[1], fy, g.MW[3]));
        const float rw = 1.0f / W;
        const float fu = __builtin_fmaf(g.MU[0], fx, __builtin_fmaf(g.MU[1], fy, g.MU[3])) * rw;
        const float fv0 = __builtin_fmaf(g.MV[2], fz0, __builtin_fmaf(g.MV[0], fx, __builtin_fmaf(g.MV[1], fy, g.MV[3]))) * rw;
        const float dfv = g.MV[2] * rw;
        const float wt = rw * rw;
        const float flu = __builtin_floorf(fu);
        const int iu = (int)flu;
        const float au = fu - flu;
        const float wu0 = (unsigned)iu < (unsigned)det.nu ? 1.0f - au : 0.0f;
        const float wu1 = (unsigned)(iu + 1) < (unsigned)det.nu ? au : 0.0f;
        if (wu0 == 0.0f && wu1 == 0.0f) continue;
        const int u0 = min(max(iu, 0), det.nu - 1), u1 = min(max(iu + 1, 0), det.nu - 1);
        const float* pk = proj + (int64_t)k * det.nv * det.nu;
#pragma unroll
        for (int z = 0; z < FDK_ZC; ++z) {
            const float fv = __builtin_fmaf((float)z, dfv, fv0);
            const float flv = __builtin_floorf(fv);
            const int iv = (int)flv;
            const float av = fv - flv;
            const float wv0 = (unsigned)iv < (unsigned)det.nv ? 1.0f - av : 0.0f;
            const float wv1 = (unsigned)(iv + 1) < (unsigned)det.nv ? av : 0.0f;
            const int v0 = min(max(iv, 0), det.nv - 1), v1 = min(max(iv + 1, 0), det.nv - 1);
            const float* r0 = pk + (int64_t)v0 * det.nu;
            const float* r1 = pk + (int64_t)v1 * det.nu;
            const float s0 = __builtin_fmaf(wu0, r0[u0], wu1 * r0[u1]);
            const float s1 = __builtin_fmaf(wu0, r1[u0], wu1 * r1[u1]);
            acc[z] = __builtin_fmaf(wt, __builtin_fmaf(wv0, s0, wv1 * s1), acc[z]);
        }
    }
#pragma unroll
    for (int z = 0; z < FDK_ZC; ++z) {
        const int iz = iz0 + z;
        if (iz >= v.nz) break;
        float* o = vol + ((int64_t)iz * v.ny + iy) * v.nx + ix;
        *o = beta == 0.0f ? acc[z] : __builtin_fmaf(beta, *o, acc[z]);
    }
}

// ------------------------------------------------------------------- filter
// Two detector rows per workgroup, packed as one complex row z = a + i b.
// With a real, even filter response H, IFFT(H . FFT(z)) = (h * a) + i (h * b).
// The forward transform is decimation-in-frequency (natural order in,
// bit-reversed out), the response is stored bit-reversed, and the inverse is
// decimation-in-time (bit-reversed in, natural out), so no permutation pass
// is needed.  The whole length-L row lives in LDS.
struct FilterArgs {
    int nu, nv;
    int L, logL;
    float DSD, du, dv, ou, ov;
    float scale;        // angular factor (pi/N or 2 pi/N)
    int wang;
    float wang_D;       // overlap half-width (mm)
    float wang_sign;    // sign of the lateral detector offset
};

__device__ __forceinline__ float2 cmul(float2 a, float2 b)
{
    return make_float2(__builtin_fmaf(a.x, b.x, -a.y * b.y), __builtin_fmaf(a.x, b.y, a.y * b.x));
}

__device__ __forceinline__ float row_weight(const FilterArgs& fa, int iu, int iv)
{
    const float u = __builtin_fmaf((float)iu + 0.5f - 0.5f * (float)fa.nu, fa.du, fa.ou);
    const float v = __builtin_fmaf((float)iv + 0.5f - 0.5f * (float)fa.nv, fa.dv, fa.ov);
    float w = fa.DSD / __builtin_sqrtf(__builtin_fmaf(fa.DSD, fa.DSD, __builtin_fmaf(u, u, v * v)));
    if (fa.wang) {
        const float up = u * fa.wang_sign;
        float ww;
        if (up >= fa.wang_D) ww = 1.0f;
        else if (up <= -fa.wang_D) ww = 0.0f;
        else {
            const float sn = __builtin_sinf(0.78539816339744830962f * (up + fa.wang_D) / fa.wang_D);
            ww = sn * sn;
        }
        w *= ww;
    }
    return w;
}

// Radix-4 passes: two consecutive radix-2 stages fused in registers, with
// the same butterflies, twiddles and rounding as the stages they replace
// (so the result is that of the radix-2 transform), half the LDS round trips
// and barriers, and the twiddle table copied to LDS when it fits (TWL).
// DIF stage pair (span S, then S/2), butterfly t < L/4: Q = S/2, j = t mod Q,
// elements b + j + {0, Q, 2Q, 3Q} with b = (t / Q) 2S.  DIT stage pair (span
// S, then 2S): j = t mod S, elements b + j + {0, S, 2S, 3S}, b = (t / S) 4S.
// An odd stage count leaves one radix-2 stage (the last DIF, the first DIT).
template <bool TWL>
__global__ void __launch_bounds__(256) k_fdk_filter(const float* in, float* out, const float* __restrict__ H,
                                                    const float2* __restrict__ twg, int64_t nrows, FilterArgs fa)
{
    extern __shared__ float2 buf[];
    const int L = fa.L, L2 = L >> 1, L4 = L >> 2;
    float2* const tws = buf + L;
    const float2* const tw = TWL ? tws : twg;
    const int64_t r0 = 2 * (int64_t)blockIdx.x, r1 = r0 + 1;
    const bool has1 = r1 < nrows;
    const int iv0 = (int)(r0 % fa.nv), iv1 = (int)(r1 % fa.nv);
    const float* a = in + r0 * fa.nu;
    const float* bb = in + r1 * fa.nu;
    for (int n = threadIdx.x; n < L; n += blockDim.x) {
        float x = 0.0f, y = 0.0f;
        if (n < fa.nu) {
            x = a[n] * row_weight(fa, n, iv0);
            if (has1) y = bb[n] * row_weight(fa, n, iv1);
        }
        buf[n] = make_float2(x, y);
    }
    if (TWL)
        for (int n = threadIdx.x; n < L2; n += blockDim.x) tws[n] = twg[n];
    __syncthreads();
    // forward DIF, stage pairs (S, S/2) from S = L/2; twiddle exp(-2 pi i j / (2 span))
    int span = L2;
    for (; span >= 2; span >>= 2) {
        const int Q = span >> 1, ts = L / (2 * span);
        for (int t = threadIdx.x; t < L4; t += blockDim.x) {
            const int j = t & (Q - 1);
            const int i0 = ((t - j) << 2) + j;   // (t / Q) 2S + j
            const float2 x0 = buf[i0], x1 = buf[i0 + Q], x2 = buf[i0 + span], x3 = buf[i0 + span + Q];
            const float2 y0 = make_float2(x0.x + x2.x, x0.y + x2.y);
            const float2 y2 = cmul(make_float2(x0.x - x2.x, x0.y - x2.y), tw[j * ts]);
            const float2 y1 = make_float2(x1.x + x3.x, x1.y + x3.y);
            const float2 y3 = cmul(make_float2(x1.x - x3.x, x1.y - x3.y), tw[(j + Q) * ts]);
            const float2 c = tw[j * 2 * ts];
            buf[i0] = make_float2(y0.x + y1.x, y0.y + y1.y);
            buf[i0 + Q] = cmul(make_float2(y0.x - y1.x, y0.y - y1.y), c);
            buf[i0 + span] = make_float2(y2.x + y3.x, y2.y + y3.y);
            buf[i0 + span + Q] = cmul(make_float2(y2.x - y3.x, y2.y - y3.y), c);
        }
        __syncthreads();
    }
    if (span == 1) {   // odd stage count: the last radix-2 stage (twiddle 1)
        for (int t = threadIdx.x; t < L2; t += blockDim.x) {
            const float2 u = buf[2 * t], w = buf[2 * t + 1];
            buf[2 * t] = make_float2(u.x + w.x, u.y + w.y);
            buf[2 * t + 1] = cmul(make_float2(u.x - w.x, u.y - w.y), tw[0]);
        }
        __syncthreads();
    }
    // response (bit-reversed order, 1/L and tau folded in) times the angular scale
    for (int n = threadIdx.x; n < L; n += blockDim.x) {
        const float h = H[n] * fa.scale;
        const float2 z = buf[n];
        buf[n] = make_float2(z.x * h, z.y * h);
    }
    __syncthreads();
    // inverse DIT; twiddle exp(+2 pi i j / (2 span)).  With an odd stage count
    // the first stage (span 1, twiddle 1) runs alone.
    span = 1;
    if (fa.logL & 1) {
        for (int t = threadIdx.x; t < L2; t += blockDim.x) {
            const float2 c = tw[0];
            const float2 w = cmul(buf[2 * t + 1], make_float2(c.x, -c.y));
            const float2 u = buf[2 * t];
            buf[2 * t] = make_float2(u.x + w.x, u.y + w.y);
            buf[2 * t + 1] = make_float2(u.x - w.x, u.y - w.y);
        }
        __syncthreads();
        span = 2;
    }
    for (; span < L; span <<= 2) {
        const int ts1 = L / (2 * span), ts2 = L / (4 * span);
        for (int t = threadIdx.x; t < L4; t += blockDim.x) {
            const int j = t & (span - 1);
            const int i0 = ((t - j) << 2) + j;   // (t / S) 4S + j
            const float2 c1 = tw[j * ts1], ca = tw[j * ts2], cb = tw[(j + span) * ts2];
            const float2 x0 = buf[i0], x1 = buf[i0 + span], x2 = buf[i0 + 2 * span], x3 = buf[i0 + 3 * span];
            const float2 w1 = cmul(x1, make_float2(c1.x, -c1.y));
            const float2 y0 = make_float2(x0.x + w1.x, x0.y + w1.y), y1 = make_float2(x0.x - w1.x, x0.y - w1.y);
            const float2 w3 = cmul(x3, make_float2(c1.x, -c1.y));
            const float2 y2 = make_float2(x2.x + w3.x, x2.y + w3.y), y3 = make_float2(x2.x - w3.x, x2.y - w3.y);
            const float2 wa = cmul(y2, make_float2(ca.x, -ca.y));
            const float2 wb = cmul(y3, make_float2(cb.x, -cb.y));
            buf[i0] = make_float2(y0.x + wa.x, y0.y + wa.y);
            buf[i0 + 2 * span] = make_float2(y0.x - wa.x, y0.y - wa.y);
            buf[i0 + span] = make_float2(y1.x + wb.x, y1.y + wb.y);
            buf[i0 + 3 * span] = make_float2(y1.x - wb.x, y1.y - wb.y);
        }
        __syncthreads();
    }
    float* oa = out + r0 * fa.nu;
    float* ob = out + r1 * fa.nu;
    for (int n = threadIdx.x; n < fa.nu; n += blockDim.x) {
        oa[n] = buf[n].x;
        if (has1) ob[n] = buf[n].y;
    }
}

}  // namespace

hipError_t launch_backward_fdk(const Plan& p, const float* proj, float* vol, int64_t view0, int64_t nviews,
                               float beta, hipStream_t s)
{
    const int nbx = (p.vol.nx + FDK_TX - 1) / FDK_TX;
    const int nby = (p.vol.ny + FDK_TY - 1) / FDK_TY;
    const int nbz = (p.vol.nz + FDK_ZC - 1) / FDK_ZC;
    const unsigned blocks = (unsigned)nbx * nby * nbz;
    hipLaunchKernelGGL(k_backward_fdk, dim3(blocks), dim3(FDK_TX * FDK_TY), 0, s, proj, vol, p.d_views,
                       (int)view0, (int)nviews, p.vol, p.det, nbx, nby, beta);
    return hipGetLastError();
}

hipError_t launch_fdk_filter(const Plan& p, int wang, const float* proj, float* out, int64_t view0, int64_t nviews,
                             hipStream_t s)
{
    (void)view0;
    const ctmi_geometry& g = p.geo;
    FilterArgs fa;
    fa.nu = p.det.nu;
    fa.nv = p.det.nv;
    fa.L = p.fft_len;
    fa.logL = p.fft_log2;
    fa.DSD = (float)g.DSD;
    fa.du = (float)g.dDetector[1];
    fa.dv = (float)g.dDetector[0];
    fa.ou = (float)g.offDetector[1];
    fa.ov = (float)g.offDetector[0];
    const double dtheta = 2.0 * 3.14159265358979323846 / (double)p.nviews;
    fa.wang = (wang && g.offDetector[1] != 0.0) ? 1 : 0;
    fa.scale = (float)(fa.wang ? dtheta : 0.5 * dtheta);
    fa.wang_D = (float)(0.5 * (double)p.det.nu * g.dDetector[1] - (g.offDetector[1] < 0 ? -g.offDetector[1] : g.offDetector[1]));
    fa.wang_sign = g.offDetector[1] < 0 ? -1.0f : 1.0f;
    const int64_t nrows = nviews * p.det.nv;
    const unsigned blocks = (unsigned)((nrows + 1) / 2);
    // the row and, up to L = 4096 (48 KB), the twiddle table in LDS
    if (p.fft_len <= 4096) {
        const size_t lds = sizeof(float2) * (size_t)(p.fft_len + p.fft_len / 2);
        hipLaunchKernelGGL(k_fdk_filter<true>, dim3(blocks), dim3(256), lds, s, proj, out, p.d_filter, p.d_twiddle,
                           nrows, fa);
    } else {
        const size_t lds = sizeof(float2) * (size_t)p.fft_len;
        hipLaunchKernelGGL(k_fdk_filter<false>, dim3(blocks), dim3(256), lds, s, proj, out, p.d_filter, p.d_twiddle,
                           nrows, fa);
    }
    return hipGetLastError();
}

}  // namespace ctmi
