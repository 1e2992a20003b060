// Diagonal of the PA operator from the stored quadrature data D.
//
// For local node I = (i,j,k) with 1-D factors B_a = B[a][i], G_a = G[a][i] (and likewise
// for j over b, k over c), the reference gradient of phi_I at (a,b,c) is
// (G_a B_b B_c, B_a G_b B_c, B_a B_b G_c), so
//   diag_e(I) = sum_{abc} sum_{mn} D_mn(abc) g_m g_n  (+ D_mass (B_a B_b B_c)^2).
// The six products of 1-D factors are formed per axis once per thread; the sum over the
// quadrature points is direct.  diag = sum_e G_e^T diag_e.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hexpa {

namespace {

template <int D, int Q, int OPS>
__global__ __launch_bounds__(256) void k_diag(int64_t nelem, const int32_t *__restrict__ emap,
                                              const double *__restrict__ qd, const DevTables *__restrict__ tab,
                                              double *__restrict__ diag)
{
    constexpr bool kMass = OPS & 1, kDiff = OPS & 2;
    constexpr int NC = kDiff ? (kMass ? 7 : 6) : 1;
    constexpr int Q3 = Q * Q * Q, D3 = D * D * D;
    __shared__ double sq[NC * Q3];
    const int64_t e = blockIdx.x;
    const double *src = qd + e * (int64_t)(NC * Q3);
    for (int t = threadIdx.x; t < NC * Q3; t += 256) sq[t] = src[t];
    __syncthreads();
    for (int I = threadIdx.x; I < D3; I += 256) {
        const int i = I % D, j = (I / D) % D, k = I / (D * D);
        double Bi[Q], Gi[Q], Bj[Q], Gj[Q], Bk[Q], Gk[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) {
            Bi[a] = tab->B[a * D + i]; Gi[a] = tab->G[a * D + i];
            Bj[a] = tab->B[a * D + j]; Gj[a] = tab->G[a * D + j];
            Bk[a] = tab->B[a * D + k]; Gk[a] = tab->G[a * D + k];
        }
        double acc = 0.0;
        for (int c = 0; c < Q; ++c)
            for (int b = 0; b < Q; ++b)
#pragma unroll
                for (int a = 0; a < Q; ++a) {
                    const int r = a + Q * (b + Q * c);
                    if constexpr (kDiff) {
                        const double g0 = Gi[a] * Bj[b] * Bk[c], g1 = Bi[a] * Gj[b] * Bk[c], g2 = Bi[a] * Bj[b] * Gk[c];
                        acc += sq[r] * g0 * g0 + sq[3 * Q3 + r] * g1 * g1 + sq[5 * Q3 + r] * g2 * g2 +
                               2.0 * (sq[Q3 + r] * g0 * g1 + sq[2 * Q3 + r] * g0 * g2 + sq[4 * Q3 + r] * g1 * g2);
                    }
                    if constexpr (kMass) {
                        const double u = Bi[a] * Bj[b] * Bk[c];
                        acc += sq[(NC - 1) * Q3 + r] * u * u;
                    }
                }
        unsafeAtomicAdd(diag + emap[e * D3 + I], acc);
    }
}

template <int P>
hipError_t launch_diag_p(const pa_op *op, double *diag, hipStream_t s)
{
    constexpr int D = P + 1;
    const dim3 grid(op->nelem), block(256);
    if (op->q == P + 1) {
        if (op->ops == 1) hipLaunchKernelGGL((k_diag<D, P + 1, 1>), grid, block, 0, s, (int64_t)op->nelem, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
        if (op->ops == 2) hipLaunchKernelGGL((k_diag<D, P + 1, 2>), grid, block, 0, s, (int64_t)op->nelem, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
        if (op->ops == 3) hipLaunchKernelGGL((k_diag<D, P + 1, 3>), grid, block, 0, s, (int64_t)op->nelem, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
    } else {
        if (op->ops == 1) hipLaunchKernelGGL((k_diag<D, P + 2, 1>), grid, block, 0, s, (int64_t)op->nelem, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
        if (op->ops == 2) hipLaunchKernelGGL((k_diag<D, P + 2, 2>), grid, block, 0, s, (int64_t)op->nelem, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
        if (op->ops == 3) hipLaunchKernelGGL((k_diag<D, P + 2, 3>), grid, block, 0, s, (int64_t)op->nelem, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_diag(const pa_op *op, double *diag, hipStream_t s)
{
    hipError_t err = vec_fill(diag, 0.0, op->ndof, s);
    if (err != hipSuccess) return err;
    switch (op->p) {
    case 1: return launch_diag_p<1>(op, diag, s);
    case 2: return launch_diag_p<2>(op, diag, s);
    case 3: return launch_diag_p<3>(op, diag, s);
    case 4: return launch_diag_p<4>(op, diag, s);
    case 5: return launch_diag_p<5>(op, diag, s);
    case 6: return launch_diag_p<6>(op, diag, s);
    case 7: return launch_diag_p<7>(op, diag, s);
    case 8: return launch_diag_p<8>(op, diag, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace hexpa
