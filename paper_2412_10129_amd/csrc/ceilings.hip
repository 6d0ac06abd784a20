// Measurement kernels: the two machine ceilings against which every
// projector, filter and vector kernel is placed (bytes moved per second of
// HBM, and non-packed FP32 vector instructions per second).  They compute
// nothing of the reconstruction; the benchmark times them on the same GPU
// right before the kernels it rates.
#include "ctmi_internal.h"

namespace ctmi {

namespace {

// Streaming copy: each workgroup copies one tile of 4 x 256 16-byte
// vectors, issuing its four loads before its four stores so that several
// requests per lane are in flight; non-temporal accesses (the data is
// touched once).
constexpr int CU4 = 4;
typedef float vf4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_stream_copy(const vf4* __restrict__ src, vf4* __restrict__ dst, int64_t n4)
{
    const int64_t base = (int64_t)blockIdx.x * (256 * CU4) + threadIdx.x;
    if (base + 256 * (CU4 - 1) < n4) {
        vf4 v[CU4];
#pragma unroll
        for (int k = 0; k < CU4; ++k) v[k] = __builtin_nontemporal_load(src + base + 256 * k);
#pragma unroll
        for (int k = 0; k < CU4; ++k) __builtin_nontemporal_store(v[k], dst + base + 256 * k);
    } else {
        for (int k = 0; k < CU4; ++k) {
            const int64_t i = base + 256 * k;
            if (i < n4) dst[i] = src[i];
        }
    }
}

// CH independent FMA chains per lane, `iters` steps each: CH * iters
// v_fma_f32 per lane (the library is built without packed FP32, so each is
// one non-packed lane-instruction).  The operands depend on the lane and on
// a run-time argument, so nothing folds; the sum is stored so nothing is
// dropped.
constexpr int CH = 16;
__global__ void __launch_bounds__(256) k_fma_loop(float* __restrict__ out, int iters, float a, float b)
{
    float c[CH];
#pragma unroll
    for (int k = 0; k < CH; ++k) c[k] = (float)(threadIdx.x + k) * 1e-3f;
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < CH; ++k) c[k] = __builtin_fmaf(c[k], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int k = 0; k < CH; ++k) s += c[k];
    out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = s;
}

}  // namespace

hipError_t launch_stream_copy(const float* src, float* dst, int64_t n, hipStream_t s)
{
    const int64_t n4 = n / 4;
    const int64_t blocks = (n4 + 256 * CU4 - 1) / (256 * CU4);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_stream_copy, dim3((unsigned)blocks), dim3(256), 0, s, reinterpret_cast<const vf4*>(src),
                       reinterpret_cast<vf4*>(dst), n4);
    return hipGetLastError();
}

int fma_loop_chains() { return CH; }

hipError_t launch_fma_loop(float* out, int blocks, int iters, hipStream_t s)
{
    hipLaunchKernelGGL(k_fma_loop, dim3((unsigned)blocks), dim3(256), 0, s, out, iters, 0.999f, 1e-4f);
    return hipGetLastError();
}

}  // namespace ctmi
