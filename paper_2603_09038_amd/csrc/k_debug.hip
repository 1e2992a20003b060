// One FP64 MFMA, for pinning the operand/lane layout the apply kernels rely on.
// Operands: A-operand lane l = A[l % 16][l / 16], B-operand lane l = B[l / 16][l % 16].
// The raw accumulator is written lane-major (Draw[4 l + v] = acc[v]) so the test can
// read off which (row, col) of D = A B each lane/element holds.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hexpa {

namespace {
typedef double dbl4 __attribute__((ext_vector_type(4)));

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
}  // namespace

hipError_t launch_debug_mfma(const double *A, const double *B, double *D, hipStream_t s)
{
    hipLaunchKernelGGL(k_debug_mfma, dim3(1), dim3(64), 0, s, A, B, D);
    return hipGetLastError();
}

}  // namespace hexpa
