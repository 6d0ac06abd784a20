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
//
// Views are taken FDK_VB at a time: the detector footprint of the
// workgroup's voxel block in each view (bounding box of its 8 projected
// corners, one pixel of margin below and two above, clamped to the
// detector) is staged in LDS with coalesced row reads, and the bilinear
// taps read LDS.  A footprint larger than FDK_CAP pixels (or a block corner
// not in front of the source) reads its view from global memory instead.
// The values read are the same either way, so the result does not depend on
// the path.
#ifndef CTMI_FDK_TX
#define CTMI_FDK_TX 32
#endif
#ifndef CTMI_FDK_ZC
#define CTMI_FDK_ZC 16
#endif
constexpr int FDK_TX = CTMI_FDK_TX, FDK_TY = 256 / FDK_TX, FDK_ZC = CTMI_FDK_ZC;
#ifndef CTMI_FDK_VB
#define CTMI_FDK_VB 2
#endif
#ifndef CTMI_FDK_CAP
#define CTMI_FDK_CAP 2560
#endif
#ifndef CTMI_FDK_P
#define CTMI_FDK_P 64
#endif
constexpr int FDK_VB = CTMI_FDK_VB, FDK_CAP = CTMI_FDK_CAP;
// Row pitch of a staged footprint up to FDK_P pixels wide: a compile-time
// pitch puts a voxel's four taps at one address plus immediate offsets
// (two paired LDS reads).
constexpr int FDK_P = CTMI_FDK_P;
static_assert(FDK_P + 1 <= 255, "paired-read offsets are 8-bit dword counts");
#ifndef CTMI_FDK_XCD
#define CTMI_FDK_XCD 0
#endif

struct FdkBox {
    int u0, v0, w, h;   // staged pixels [u0, u0 + w) x [v0, v0 + h); w = 0: not staged
    int pitch;          // LDS row pitch (floats): FDK_P when w <= FDK_P and it fits, else w
    float rw;           // 1 / w
    int inner;          // pitch FDK_P and no margin clipped by the detector (below)
};

#ifndef CTMI_FDK_WAVES
#define CTMI_FDK_WAVES 6
#endif
__global__ void __launch_bounds__(FDK_TX* FDK_TY) __attribute__((amdgpu_waves_per_eu(CTMI_FDK_WAVES, 8))) k_backward_fdk(const float* __restrict__ proj,
                                                                 float* __restrict__ vol,
                                                                 const ViewGeo* __restrict__ tab, int view0,
                                                                 int nviews, VolDims v, DetDims det, int nbx,
                                                                 int nby, float beta)
{
    __shared__ float box[FDK_VB][FDK_CAP];
    __shared__ FdkBox fb[FDK_VB];
    const int b = CTMI_FDK_XCD ? (int)xcd_contiguous(blockIdx.x, gridDim.x) : (int)blockIdx.x;
    const int bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
    const int ix = bx * FDK_TX + (int)(threadIdx.x % FDK_TX);
    const int iy = by * FDK_TY + (int)(threadIdx.x / FDK_TX);
    const int iz0 = bz * FDK_ZC;
    const bool live = ix < v.nx && iy < v.ny;   // every thread takes part in staging
    // the block's voxel centres (clamped to the volume)
    const float lo[3] = {(float)(bx * FDK_TX), (float)(by * FDK_TY), (float)iz0};
    const float hi[3] = {(float)(min((bx + 1) * FDK_TX, v.nx) - 1), (float)(min((by + 1) * FDK_TY, v.ny) - 1),
                         (float)(min(iz0 + FDK_ZC, v.nz) - 1)};
    const float fx = (float)ix, fy = (float)iy, fz0 = (float)iz0;
    float acc[FDK_ZC];
#pragma unroll
    for (int z = 0; z < FDK_ZC; ++z) acc[z] = 0.0f;

    for (int k0 = 0; k0 < nviews; k0 += FDK_VB) {
        const int nb = min(FDK_VB, nviews - k0);
        __syncthreads();   // the previous chunk's reads of box and fb are done
        if ((int)threadIdx.x < nb) {
            const ViewGeo& g = tab[view0 + k0 + threadIdx.x];
            float umin = CTMI_INF, umax = -CTMI_INF, vmin = CTMI_INF, vmax = -CTMI_INF, wmin = CTMI_INF;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const float cx = (q & 1) ? hi[0] : lo[0], cy = (q & 2) ? hi[1] : lo[1], cz = (q & 4) ? hi[2] : lo[2];
                const float W = __builtin_fmaf(g.MW[0], cx, __builtin_fmaf(g.MW[1], cy, __builtin_fmaf(g.MW[2], cz, g.MW[3])));
                const float U = __builtin_fmaf(g.MU[0], cx, __builtin_fmaf(g.MU[1], cy, __builtin_fmaf(g.MU[2], cz, g.MU[3])));
                const float V = __builtin_fmaf(g.MV[0], cx, __builtin_fmaf(g.MV[1], cy, __builtin_fmaf(g.MV[2], cz, g.MV[3])));
                const float rw = 1.0f / W;
                wmin = fminf(wmin, W);
                umin = fminf(umin, U * rw);
                umax = fmaxf(umax, U * rw);
                vmin = fminf(vmin, V * rw);
                vmax = fmaxf(vmax, V * rw);
            }
            FdkBox f;
            f.w = 0;
            f.u0 = f.v0 = f.h = 0;
            f.pitch = 0;
            f.rw = 1.0f;
            f.inner = 0;
            // clamp in float first: corners may project far off the detector
            umin = fminf(fmaxf(umin, -4.0f), (float)det.nu + 4.0f);
            umax = fminf(fmaxf(umax, -4.0f), (float)det.nu + 4.0f);
            vmin = fminf(fmaxf(vmin, -4.0f), (float)det.nv + 4.0f);
            vmax = fminf(fmaxf(vmax, -4.0f), (float)det.nv + 4.0f);
            const int u0 = max((int)__builtin_floorf(umin) - 1, 0), u1 = min((int)__builtin_floorf(umax) + 2, det.nu - 1);
            const int v0 = max((int)__builtin_floorf(vmin) - 1, 0), v1 = min((int)__builtin_floorf(vmax) + 2, det.nv - 1);
            // a voxel of the block projects inside the corners' bounding
            // box (all in front of the source; on a circular orbit u does
            // not depend on z), so its taps floor(u), floor(u) + 1 lie in
            // [floor(umin) - 1, floor(umax) + 2], and the same for v, with a
            // pixel to spare for rounding: when no end was clipped, every tap
            // is on the detector and in the box.  (A block cut by the
            // volume's last z plane still runs its threads past it, outside
            // [lo, hi]: it keeps the clamped taps.)
            const bool inner = (int)__builtin_floorf(vmin) - 1 >= 0 && (int)__builtin_floorf(vmax) + 2 <= det.nv - 1 &&
                               (int)__builtin_floorf(umin) - 1 >= 0 && (int)__builtin_floorf(umax) + 2 <= det.nu - 1 &&
                               iz0 + FDK_ZC <= v.nz;
            // (each side is checked first, so the product cannot overflow)
            if (wmin > 0.0f && u0 <= u1 && v0 <= v1 && u1 - u0 < FDK_CAP && v1 - v0 < FDK_CAP) {
                const int w = u1 - u0 + 1, h = v1 - v0 + 1;
                const int pitch = w <= FDK_P && h * FDK_P <= FDK_CAP ? FDK_P : w;
                if (h * pitch <= FDK_CAP) {
                    f.u0 = u0;
                    f.v0 = v0;
                    f.w = w;
                    f.h = h;
                    f.pitch = pitch;
                    f.rw = 1.0f / (float)w;
                    f.inner = inner && pitch == FDK_P ? 1 : 0;
                }
            }
            fb[threadIdx.x] = f;
        }
        __syncthreads();
        for (int q = 0; q < nb; ++q) {
            const FdkBox f = fb[q];
            if (f.w == 0) continue;
            const float* pk = proj + (int64_t)(k0 + q) * det.nv * det.nu;
            const int n = f.w * f.h;
            for (int i = threadIdx.x; i < n; i += blockDim.x) {
                // row i / w from FP32 ((i + 1/2) / w is at least 1/(2w) from an integer)
                const int r = (int)(((float)i + 0.5f) * f.rw);
                box[q][r * f.pitch + (i - r * f.w)] = pk[(int64_t)(f.v0 + r) * det.nu + f.u0 + (i - r * f.w)];
            }
        }
        __syncthreads();
        if (!live) continue;
        for (int q = 0; q < nb; ++q) {
            const int k = k0 + q;
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
            const FdkBox f = fb[q];
            if (f.w > 0) {
                // staged: LDS offsets clamped into the box (a no-op when the
                // footprint holds the taps, which its margins ensure); the
                // columns once per view, the rows per voxel unless the box
                // holds every row the block can tap
                const int c0 = min(max(u0 - f.u0, 0), f.w - 1), c1 = min(max(u1 - f.u0, 0), f.w - 1);
                const float* bq = box[q];
                if (f.inner) {
                    // every tap lies in the box and on the detector (above):
                    // no clamps and no zero weights (wu0, wu1 are 1 - au, au);
                    // the row offset is an exact FP32 integer (below 2^24)
                    const float v0f = (float)f.v0;
                    const float* b = bq + (iu - f.u0);
#pragma unroll
                    for (int z = 0; z < FDK_ZC; ++z) {
                        const float fv = __builtin_fmaf((float)z, dfv, fv0);
                        const float flv = __builtin_floorf(fv);
                        const float av = fv - flv;
                        const float* t = b + (int)((flv - v0f) * (float)FDK_P);
                        const float s0 = __builtin_fmaf(wu0, t[0], wu1 * t[1]);
                        const float s1 = __builtin_fmaf(wu0, t[FDK_P], wu1 * t[FDK_P + 1]);
                        acc[z] = __builtin_fmaf(wt, __builtin_fmaf(1.0f - av, s0, av * s1), acc[z]);
                    }
                    continue;
                }
#pragma unroll
                for (int z = 0; z < FDK_ZC; ++z) {
                    const float fv = __builtin_fmaf((float)z, dfv, fv0);
                    const float flv = __builtin_floorf(fv);
                    const int iv = (int)flv;
                    const float av = fv - flv;
                    const float wv0 = (unsigned)iv < (unsigned)det.nv ? 1.0f - av : 0.0f;
                    const float wv1 = (unsigned)(iv + 1) < (unsigned)det.nv ? av : 0.0f;
                    const int r0 = min(max(min(max(iv, 0), det.nv - 1) - f.v0, 0), f.h - 1);
                    const int r1 = min(max(min(max(iv + 1, 0), det.nv - 1) - f.v0, 0), f.h - 1);
                    const float* p0 = bq + r0 * f.pitch;
                    const float* p1 = bq + r1 * f.pitch;
                    const float s0 = __builtin_fmaf(wu0, p0[c0], wu1 * p0[c1]);
                    const float s1 = __builtin_fmaf(wu0, p1[c0], wu1 * p1[c1]);
                    acc[z] = __builtin_fmaf(wt, __builtin_fmaf(wv0, s0, wv1 * s1), acc[z]);
                }
            } else {
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
        }
    }
    if (!live) return;
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

// Detector row iv's constant in the cosine weight: DSD^2 + v^2.
__device__ __forceinline__ float row_const(const FilterArgs& fa, int iv)
{
    const float v = __builtin_fmaf((float)iv + 0.5f - 0.5f * (float)fa.nv, fa.dv, fa.ov);
    return __builtin_fmaf(fa.DSD, fa.DSD, v * v);
}

// Pre-weight of pixel (iu, row with constant cv): DSD / sqrt(DSD^2 + u^2 +
// v^2) with the hardware reciprocal square root (1 ulp), times Wang's
// offset-detector weight when asked for.
__device__ __forceinline__ float row_weight(const FilterArgs& fa, int iu, float cv)
{
    const float u = __builtin_fmaf((float)iu + 0.5f - 0.5f * (float)fa.nu, fa.du, fa.ou);
    float w = fa.DSD * __builtin_amdgcn_rsqf(__builtin_fmaf(u, u, cv));
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

// LDS slot of row element i: one float2 of padding per 16 (P) breaks the
// power-of-two strides of the small-span passes across the LDS banks.
template <bool P>
__device__ __forceinline__ int pad(int i) { return P ? i + (i >> 4) : i; }

// LDS slot of row element i for the compile-time lengths: bits 5-7 of i
// are XORed into bits 2-4 and 0-2 (a permutation within each 32-element
// block), which spreads the strided and the contiguous small-span accesses
// over the banks without padding.
#ifndef CTMI_FILTER_SWZ
#define CTMI_FILTER_SWZ 1
#endif
__device__ __forceinline__ int swz(int i)
{
    const int g = (i >> 5) & 7;
    return i ^ (g << 2) ^ g;
}

__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 conj2(float2 a) { return make_float2(a.x, -a.y); }

// Consecutive radix-2 stages are fused into radix-8 (three stages) and
// radix-4 (two) passes in registers, with the same butterflies, twiddles and
// rounding as the stages they replace, so the result is that of the
// radix-2 transform with a third of its LDS round trips and barriers.
// tw[k] = exp(-2 pi i k / L), k < L/2; a radix-2 stage of span S uses
// tw[j L / (2 S)] for the pair at offset j of its block.
//
// Each pass reads its inputs through `ld(i)` and writes its outputs through
// `st(i, v)` (i the row position), so the first forward pass can read the
// weighted detector row straight from global memory, the last forward pass
// can apply the filter response as it stores, and the last inverse pass can
// write the filtered row straight to global memory.
//
// DIF pass over stages S, S/2, S/4 (E = S/4): butterfly t < L/8 takes
// elements i0 + k E, k < 8, i0 = (t / E) 2S + t mod E.
//
// With Z (the first pass, S = L/2) the upper half of the row is the zero
// padding (L >= 2 nu - 1), so inputs k >= 4 are not read and the first
// stage's sums and differences are the inputs themselves.
template <bool Z = false, class LD, class ST>
__device__ __forceinline__ void dif8(const float2* tw, int L, int S, int t0, int dt, LD ld, ST st)
{
    const int E = S >> 2, ts1 = L / (2 * S);
    for (int t = t0; t < (L >> 3); t += dt) {
        const int j = t & (E - 1);
        const int i0 = ((t - j) << 3) + j;
        float2 x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = (Z && k >= 4) ? make_float2(0.0f, 0.0f) : ld(i0 + k * E);
        float2 y[8];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            y[k] = Z ? x[k] : cadd(x[k], x[k + 4]);
            y[k + 4] = cmul(Z ? x[k] : csub(x[k], x[k + 4]), tw[(j + k * E) * ts1]);
        }
        const float2 c0 = tw[j * 2 * ts1], c1 = tw[(j + E) * 2 * ts1], c3 = tw[j * 4 * ts1];
#pragma unroll
        for (int q = 0; q < 8; q += 4) {
            const float2 z0 = cadd(y[q], y[q + 2]), z2 = cmul(csub(y[q], y[q + 2]), c0);
            const float2 z1 = cadd(y[q + 1], y[q + 3]), z3 = cmul(csub(y[q + 1], y[q + 3]), c1);
            st(i0 + q * E, cadd(z0, z1));
            st(i0 + (q + 1) * E, cmul(csub(z0, z1), c3));
            st(i0 + (q + 2) * E, cadd(z2, z3));
            st(i0 + (q + 3) * E, cmul(csub(z2, z3), c3));
        }
    }
}

// DIF pass over stages S, S/2 (Q = S/2): elements i0 + {0, Q, 2Q, 3Q},
// i0 = (t / Q) 2S + t mod Q.
template <class LD, class ST>
__device__ __forceinline__ void dif4(const float2* tw, int L, int S, int t0, int dt, LD ld, ST st)
{
    const int Q = S >> 1, ts = L / (2 * S);
    for (int t = t0; t < (L >> 2); t += dt) {
        const int j = t & (Q - 1);
        const int i0 = ((t - j) << 2) + j;
        const float2 x0 = ld(i0), x1 = ld(i0 + Q), x2 = ld(i0 + S), x3 = ld(i0 + S + Q);
        const float2 y0 = cadd(x0, x2), y2 = cmul(csub(x0, x2), tw[j * ts]);
        const float2 y1 = cadd(x1, x3), y3 = cmul(csub(x1, x3), tw[(j + Q) * ts]);
        const float2 c = tw[j * 2 * ts];
        st(i0, cadd(y0, y1));
        st(i0 + Q, cmul(csub(y0, y1), c));
        st(i0 + S, cadd(y2, y3));
        st(i0 + S + Q, cmul(csub(y2, y3), c));
    }
}

// DIF stage of span 1 (twiddle tw[0]).
template <class LD, class ST>
__device__ __forceinline__ void dif2(const float2* tw, int L, int t0, int dt, LD ld, ST st)
{
    for (int t = t0; t < (L >> 1); t += dt) {
        const float2 u = ld(2 * t), w = ld(2 * t + 1);
        st(2 * t, cadd(u, w));
        st(2 * t + 1, cmul(csub(u, w), tw[0]));
    }
}

// DIT pass over stages S, 2S, 4S: elements i0 + k S, k < 8,
// i0 = (t / S) 8S + t mod S.  With H (the last pass, S = L/8) only the
// lower half of the row is stored: the upper half is the padding's share of
// the circular convolution, which the filtered row does not keep.
template <bool H = false, class LD, class ST>
__device__ __forceinline__ void dit8(const float2* tw, int L, int S, int t0, int dt, LD ld, ST st)
{
    const int ts1 = L / (2 * S);
    for (int t = t0; t < (L >> 3); t += dt) {
        const int j = t & (S - 1);
        const int i0 = ((t - j) << 3) + j;
        float2 x[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = ld(i0 + k * S);
        const float2 c1 = conj2(tw[j * ts1]);
        float2 y[8];
#pragma unroll
        for (int k = 0; k < 8; k += 2) {
            const float2 w = cmul(x[k + 1], c1);
            y[k] = cadd(x[k], w);
            y[k + 1] = csub(x[k], w);
        }
        const float2 ca = conj2(tw[j * (ts1 >> 1)]), cb = conj2(tw[(j + S) * (ts1 >> 1)]);
        float2 z[8];
#pragma unroll
        for (int q = 0; q < 8; q += 4) {
            const float2 wa = cmul(y[q + 2], ca), wb = cmul(y[q + 3], cb);
            z[q] = cadd(y[q], wa);
            z[q + 2] = csub(y[q], wa);
            z[q + 1] = cadd(y[q + 1], wb);
            z[q + 3] = csub(y[q + 1], wb);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float2 w = cmul(z[k + 4], conj2(tw[(j + k * S) * (ts1 >> 2)]));
            st(i0 + k * S, cadd(z[k], w));
            if (!H) st(i0 + (k + 4) * S, csub(z[k], w));
        }
    }
}

// DIT pass over stages S, 2S: elements i0 + {0, S, 2S, 3S}, i0 = (t / S) 4S + t mod S.
template <class LD, class ST>
__device__ __forceinline__ void dit4(const float2* tw, int L, int S, int t0, int dt, LD ld, ST st)
{
    const int ts1 = L / (2 * S), ts2 = ts1 >> 1;
    for (int t = t0; t < (L >> 2); t += dt) {
        const int j = t & (S - 1);
        const int i0 = ((t - j) << 2) + j;
        const float2 c1 = conj2(tw[j * ts1]), ca = conj2(tw[j * ts2]), cb = conj2(tw[(j + S) * ts2]);
        const float2 x0 = ld(i0), x1 = ld(i0 + S), x2 = ld(i0 + 2 * S), x3 = ld(i0 + 3 * S);
        const float2 w1 = cmul(x1, c1), w3 = cmul(x3, c1);
        const float2 y0 = cadd(x0, w1), y1 = csub(x0, w1), y2 = cadd(x2, w3), y3 = csub(x2, w3);
        const float2 wa = cmul(y2, ca), wb = cmul(y3, cb);
        st(i0, cadd(y0, wa));
        st(i0 + 2 * S, csub(y0, wa));
        st(i0 + S, cadd(y1, wb));
        st(i0 + 3 * S, csub(y1, wb));
    }
}

// DIT stage of span 1 (twiddle conj(tw[0])).
template <class LD, class ST>
__device__ __forceinline__ void dit2(const float2* tw, int L, int t0, int dt, LD ld, ST st)
{
    for (int t = t0; t < (L >> 1); t += dt) {
        const float2 w = cmul(ld(2 * t + 1), conj2(tw[0]));
        const float2 u = ld(2 * t);
        st(2 * t, cadd(u, w));
        st(2 * t + 1, csub(u, w));
    }
}

// Workgroups are persistent over row pairs: each copies the twiddle table
// to LDS once (when it fits, TWL) and then filters row pairs.  LOGL > 0
// fixes the row length L = 2^LOGL at compile time (spans, twiddle strides
// and the pass schedule become constants); LOGL = 0 takes it from the
// arguments.  A pair takes TPP threads (one radix-8 butterfly each, at most
// 256), so a workgroup holds 256 / TPP pairs, each in its own LDS row; pairs
// g PPB + sub, g = blockIdx.x, blockIdx.x + gridDim.x, ...
template <int LOGL>
struct FilterShape {
    static constexpr int TPP = LOGL == 0 ? 256 : ((1 << LOGL) / 8 < 256 ? (1 << LOGL) / 8 : 256);
    static constexpr int PPB = 256 / TPP;
};

template <int LOGL, bool TWL, bool P = TWL>
__global__ void __launch_bounds__(256) k_fdk_filter(const float* in, float* out, const float* __restrict__ H,
                                                    const float2* __restrict__ twg, int64_t nrows, FilterArgs fa)
{
    static_assert(LOGL == 0 || LOGL >= 6, "fixed lengths give every thread a butterfly");
    constexpr int TPP = FilterShape<LOGL>::TPP, PPB = FilterShape<LOGL>::PPB;
    extern __shared__ float2 buf[];
    const int L = LOGL ? 1 << LOGL : fa.L, L2 = L >> 1, logL = LOGL ? LOGL : fa.logL;
    constexpr bool SWZ = LOGL > 0 && CTMI_FILTER_SWZ != 0;
    const int rowsz = L + (P && !SWZ ? L >> 4 : 0);
    float2* const tws = buf + PPB * rowsz;
    const float2* const tw = TWL ? tws : twg;
    if (TWL)
        for (int n = threadIdx.x; n < L2; n += blockDim.x) tws[n] = twg[n];
    const int sub = PPB > 1 ? (int)threadIdx.x / TPP : 0;
    const int t0 = PPB > 1 ? (int)threadIdx.x % TPP : (int)threadIdx.x;
    const int dt = PPB > 1 ? TPP : (int)blockDim.x;
    float2* const row = buf + sub * rowsz;
    auto slot = [&](int i) { return SWZ ? swz(i) : pad<P>(i); };
    auto lds_ld = [&](int i) { return row[slot(i)]; };
    auto lds_st = [&](int i, float2 v) { row[slot(i)] = v; };
    // the response (bit-reversed order, 1/L and tau folded in) times the
    // angular scale, applied as the last forward pass stores
    auto resp_st = [&](int i, float2 v) {
        const float h = H[i] * fa.scale;
        row[slot(i)] = make_float2(v.x * h, v.y * h);
    };
    const int64_t npairs = (nrows + 1) / 2;
    for (int64_t g = blockIdx.x; g * PPB < npairs; g += gridDim.x) {
        const int64_t pr = g * PPB + sub;
        const bool live = pr < npairs;   // the last group may be partial
        const int64_t r0 = 2 * pr, r1 = r0 + 1;
        const bool has1 = live && r1 < nrows;
        const int iv0 = (int)(r0 % fa.nv);
        const int iv1 = iv0 + 1 == fa.nv ? 0 : iv0 + 1;
        const float* a = in + r0 * fa.nu;
        const float* bb = in + r1 * fa.nu;
        float* oa = out + r0 * fa.nu;
        float* ob = out + r1 * fa.nu;
        // weighted rows, zero beyond nu (the linear convolution's padding)
        const float cv0 = row_const(fa, iv0), cv1 = row_const(fa, iv1);
        auto src = [&](int n) {
            float x = 0.0f, y = 0.0f;
            if (live && n < fa.nu) {
                x = a[n] * row_weight(fa, n, cv0);
                if (has1) y = bb[n] * row_weight(fa, n, cv1);
            }
            return make_float2(x, y);
        };
        auto dst = [&](int n, float2 v) {
            if (live && n < fa.nu) {
                oa[n] = v.x;
                if (has1) ob[n] = v.y;
            }
        };
        __syncthreads();   // the previous pairs are done with buf (and the twiddles are in)
        if (LOGL > 0) {
            // the last forward pass, the response and the first inverse pass
            // act on the same G = 2, 4 or 8 consecutive elements per
            // butterfly, so they run as one pass in registers (same
            // arithmetic, one LDS round trip and one barrier fewer)
            constexpr int R = LOGL % 3, G = R == 0 ? 8 : (R == 1 ? 2 : 4);
            dif8<true>(tw, L, L2, t0, dt, src, lds_st);
            __syncthreads();
            for (int span = L2 >> 3; span > G / 2; span >>= 3) {
                dif8(tw, L, span, t0, dt, lds_ld, lds_st);
                __syncthreads();
            }
            for (int t = t0; t < L / G; t += dt) {
                float2 r[G];
#pragma unroll
                for (int k = 0; k < G; ++k) r[k] = lds_ld(G * t + k);
                auto rl = [&](int i) { return r[i & (G - 1)]; };
                auto rs = [&](int i, float2 v) { r[i & (G - 1)] = v; };
                auto rr = [&](int i, float2 v) {
                    const float h = H[i] * fa.scale;
                    r[i & (G - 1)] = make_float2(v.x * h, v.y * h);
                };
                if (G == 2) {
                    dif2(tw, L, t, L, rl, rr);
                    dit2(tw, L, t, L, rl, rs);
                } else if (G == 4) {
                    dif4(tw, L, 2, t, L, rl, rr);
                    dit4(tw, L, 1, t, L, rl, rs);
                } else {
                    dif8(tw, L, 4, t, L, rl, rr);
                    dit8(tw, L, 1, t, L, rl, rs);
                }
#pragma unroll
                for (int k = 0; k < G; ++k) lds_st(G * t + k, r[k]);
            }
            __syncthreads();
            int span = G;
            for (; span < (L >> 3); span <<= 3) {
                dit8(tw, L, span, t0, dt, lds_ld, lds_st);
                __syncthreads();
            }
            dit8<true>(tw, L, span, t0, dt, lds_ld, dst);
        } else if (logL >= 3) {
            // forward DIF from span L/2: radix-8 passes, then the one or two
            // stages left; the first reads the rows, the last applies the response
            int span = L2, rem = logL;
            if (rem == 3) dif8<true>(tw, L, span, t0, dt, src, resp_st);
            else dif8<true>(tw, L, span, t0, dt, src, lds_st);
            __syncthreads();
            for (rem -= 3, span >>= 3; rem >= 3; rem -= 3, span >>= 3) {
                if (rem == 3) dif8(tw, L, span, t0, dt, lds_ld, resp_st);
                else dif8(tw, L, span, t0, dt, lds_ld, lds_st);
                __syncthreads();
            }
            if (rem == 2) {
                dif4(tw, L, span, t0, dt, lds_ld, resp_st);
                __syncthreads();
            } else if (rem == 1) {
                dif2(tw, L, t0, dt, lds_ld, resp_st);
                __syncthreads();
            }
            // inverse DIT from span 1: the one or two stages left over first,
            // then radix-8 passes; the last (span L/8) writes the rows out
            span = 1;
            rem = logL % 3;
            if (rem == 1) {
                dit2(tw, L, t0, dt, lds_ld, lds_st);
                __syncthreads();
                span = 2;
            } else if (rem == 2) {
                dit4(tw, L, 1, t0, dt, lds_ld, lds_st);
                __syncthreads();
                span = 4;
            }
            for (; span < (L >> 3); span <<= 3) {
                dit8(tw, L, span, t0, dt, lds_ld, lds_st);
                __syncthreads();
            }
            dit8<true>(tw, L, span, t0, dt, lds_ld, dst);
        } else {
            // L = 2 or 4: one load pass, the stages, the response, the store
            for (int n = t0; n < L; n += dt) lds_st(n, src(n));
            __syncthreads();
            if (logL == 2) dif4(tw, L, L2, t0, dt, lds_ld, resp_st);
            else dif2(tw, L, t0, dt, lds_ld, resp_st);
            __syncthreads();
            if (logL == 2) dit4(tw, L, 1, t0, dt, lds_ld, lds_st);
            else dit2(tw, L, t0, dt, lds_ld, lds_st);
            __syncthreads();
            for (int n = t0; n < L; n += dt) dst(n, lds_ld(n));
        }
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
    const int64_t npairs = (nrows + 1) / 2;
    // persistent workgroups: enough for 8 per CU, each looping over row pairs
    auto groups = [&](int ppb) { return (unsigned)std::min<int64_t>((npairs + ppb - 1) / ppb, 2048); };
    // up to L = 4096 the padded rows and the twiddle table in LDS (51 KB)
    const size_t row = (size_t)p.fft_len + (size_t)(p.fft_len >> 4);   // padded row
    const size_t tws = (size_t)p.fft_len / 2;
    auto fixed = [&](auto kern, int ppb) {
        const size_t frow = CTMI_FILTER_SWZ ? (size_t)p.fft_len : row;   // swizzled rows need no padding
        const size_t lds = sizeof(float2) * ((size_t)ppb * frow + tws);
        hipLaunchKernelGGL(kern, dim3(groups(ppb)), dim3(256), lds, s, proj, out, p.d_filter, p.d_twiddle, nrows,
                           fa);
    };
    switch (p.fft_log2) {
    case 9: fixed(k_fdk_filter<9, true>, FilterShape<9>::PPB); break;
    case 10: fixed(k_fdk_filter<10, true>, FilterShape<10>::PPB); break;
    case 11: fixed(k_fdk_filter<11, true>, FilterShape<11>::PPB); break;
    case 12: fixed(k_fdk_filter<12, true>, FilterShape<12>::PPB); break;
    default:
        if (p.fft_len <= 4096) {
            const size_t lds = sizeof(float2) * (row + tws);
            hipLaunchKernelGGL((k_fdk_filter<0, true>), dim3(groups(1)), dim3(256), lds, s, proj, out, p.d_filter,
                               p.d_twiddle, nrows, fa);
        } else {   // L = 8192: the unpadded row alone fills 64 KB
            const size_t lds = sizeof(float2) * (size_t)p.fft_len;
            hipLaunchKernelGGL((k_fdk_filter<0, false>), dim3(groups(1)), dim3(256), lds, s, proj, out, p.d_filter,
                               p.d_twiddle, nrows, fa);
        }
    }
    return hipGetLastError();
}

}  // namespace ctmi
