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

__global__ void __launch_bounds__(256) k_fdk_filter(const float* in, float* out, const float* __restrict__ H,
                                                    const float2* __restrict__ tw, int64_t nrows, FilterArgs fa)
{
    extern __shared__ float2 buf[];
    const int L = fa.L;
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
    __syncthreads();
    // forward DIF: spans L/2, L/4, ..., 1; twiddle exp(-2 pi i j / (2 span))
    for (int span = L >> 1, tstride = 1; span >= 1; span >>= 1, tstride <<= 1) {
        for (int t = threadIdx.x; t < (L >> 1); t += blockDim.x) {
            const int j = t & (span - 1);
            const int i0 = ((t - j) << 1) + j;
            const int i1 = i0 + span;
            const float2 u = buf[i0], w = buf[i1];
            buf[i0] = make_float2(u.x + w.x, u.y + w.y);
            buf[i1] = cmul(make_float2(u.x - w.x, u.y - w.y), tw[j * tstride]);
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
    // inverse DIT: spans 1, 2, ..., L/2; twiddle exp(+2 pi i j / (2 span))
    for (int span = 1, tstride = L >> 1; span < L; span <<= 1, tstride >>= 1) {
        for (int t = threadIdx.x; t < (L >> 1); t += blockDim.x) {
            const int j = t & (span - 1);
            const int i0 = ((t - j) << 1) + j;
            const int i1 = i0 + span;
            const float2 c = tw[j * tstride];
            const float2 w = cmul(buf[i1], make_float2(c.x, -c.y));
            const float2 u = buf[i0];
            buf[i0] = make_float2(u.x + w.x, u.y + w.y);
            buf[i1] = make_float2(u.x - w.x, u.y - w.y);
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
    const size_t lds = sizeof(float2) * (size_t)p.fft_len;
    hipLaunchKernelGGL(k_fdk_filter, dim3(blocks), dim3(256), lds, s, proj, out, p.d_filter, p.d_twiddle, nrows, fa);
    return hipGetLastError();
}

}  // namespace ctmi
