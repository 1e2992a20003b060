// One FP64 MFMA, for pinning the operand/lane layouts the apply kernels rely on.
//  shape 16: v_mfma_f64_16x16x4f64, A-operand lane l = A[l % 16][l / 16], B-operand lane
//            l = B[l / 16][l % 16]; raw accumulator written lane-major, Draw[4 l + v].
//  shape 4:  v_mfma_f64_4x4x4f64 (4 blocks), block beta = (l >> 2) & 3 takes A-operand
//            A[beta][l & 3][l >> 4] and B-operand B[beta][l >> 4][l & 3]; Draw[l] = result.
// The tests read off which entry of the product each lane/element holds.
#include <hip/hip_runtime.h>

#include "apply_common.h"

namespace hexpa {

namespace {

__global__ __launch_bounds__(64) void k_debug_mfma(const double *__restrict__ A, const double *__restrict__ B,
                                                   double *__restrict__ Draw)
{
    const int l = threadIdx.x;
    const double a = A[(l % 16) * 4 + l / 16];
    const double b = B[(l / 16) * 16 + l % 16];
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
#pragma unroll
    for (int v = 0; v < 4; ++v) Draw[4 * l + v] = acc[v];
}

__global__ __launch_bounds__(64) void k_debug_mfma4(const double *__restrict__ A, const double *__restrict__ B,
                                                    double *__restrict__ Draw)
{
    const int l = threadIdx.x, beta = (l >> 2) & 3;
    const double a = A[beta * 16 + (l & 3) * 4 + (l >> 4)];
    const double b = B[beta * 16 + (l >> 4) * 4 + (l & 3)];
    Draw[l] = __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, 0.0, 0, 0, 0);
}

// v_mfma_f32_16x16x16{f16,bf16}: lane l supplies A[l%16][4(l/16)+t], B[4(l/16)+t][l%16].
// The operands go through the apply kernels' own rounding (Mfma16<BF>::pack) and MFMA.
template <bool BF>
__global__ __launch_bounds__(64) void k_debug_mfma16(const float *__restrict__ A, const float *__restrict__ B,
                                                     float *__restrict__ Draw)
{
    const int l = threadIdx.x;
    float fa[4], fb[4];
    for (int t = 0; t < 4; ++t) {
        fa[t] = A[(l % 16) * 16 + 4 * (l / 16) + t];
        fb[t] = B[(4 * (l / 16) + t) * 16 + l % 16];
    }
    const flt4_t acc = Mfma16<BF>::mma(Mfma16<BF>::pack(fa), Mfma16<BF>::pack(fb), flt4_t{0.f, 0.f, 0.f, 0.f});
    for (int v = 0; v < 4; ++v) Draw[4 * l + v] = acc[v];
}
}  // namespace

hipError_t launch_debug_mfma16(int bf, const float *A, const float *B, float *D, hipStream_t s)
{
    if (bf)
        hipLaunchKernelGGL(k_debug_mfma16<true>, dim3(1), dim3(64), 0, s, A, B, D);
    else
        hipLaunchKernelGGL(k_debug_mfma16<false>, dim3(1), dim3(64), 0, s, A, B, D);
    return hipGetLastError();
}

hipError_t launch_debug_mfma(int shape, const double *A, const double *B, double *D, hipStream_t s)
{
    if (shape == 4)
        hipLaunchKernelGGL(k_debug_mfma4, dim3(1), dim3(64), 0, s, A, B, D);
    else
        hipLaunchKernelGGL(k_debug_mfma, dim3(1), dim3(64), 0, s, A, B, D);
    return hipGetLastError();
}

}  // namespace hexpa
