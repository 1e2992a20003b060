// Diagonal of the PA operator from the stored quadrature data D, by sum factorization.
//
// For local node I = (i,j,k) the reference gradient of phi_I at quadrature point (a,b,c)
// is g = (G_a^i B_b^j B_c^k, B_a^i G_b^j B_c^k, B_a^i B_b^j G_c^k) (B, G: 1-D basis values
// and derivatives), so
//   diag_e(I) = sum_{abc} [ sum_{mn} D_mn(abc) g_m g_n + D_mass(abc) (B_a^i B_b^j B_c^k)^2 ].
// Every term is a product of three 1-D factors taken from the per-axis tables
// B^2, BG = B G and G^2 ([Q][d] each): D_00 G^2 x B^2 x B^2, D_01 2 BG x BG x B^2,
// D_02 2 BG x B^2 x BG, D_11 B^2 x G^2 x B^2, D_12 2 B^2 x BG x BG, D_22 B^2 x B^2 x G^2,
// D_mass B^2 x B^2 x B^2.  So the diagonal is three one-index contractions, axis by axis:
//   a:  U_t(i,b,c) = sum_a X_t[a][i] D_t(a,b,c)          (one per stored component t)
//   b:  V_z(i,j,c) = sum_b sum_{t: z-table z} Y_t[b][j] U_t(i,b,c)   (terms grouped by
//       their third-axis table z in {B^2, BG, G^2}, the factors 2 folded in here)
//   c:  diag_e(i,j,k) = sum_c sum_z Z_z[c][k] V_z(i,j,c)
// at O(Q^3 d + Q^2 d^2 + Q d^3) per element instead of O(d^3 Q^3).  diag = sum_e G_e^T diag_e.
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hexpa {

namespace {

constexpr int kDiagThreads = 512;

// per-axis table index of each stored component (D order 00, 01, 02, 11, 12, 22, mass)
enum : int { T_B2 = 0, T_BG = 1, T_G2 = 2 };

template <int D, int Q, int OPS>
__global__ __launch_bounds__(kDiagThreads) void k_diag(int64_t nelem, const int32_t *__restrict__ emap,
                                                       const double *__restrict__ qd,
                                                       const DevTables *__restrict__ tab, double *__restrict__ diag)
{
    constexpr bool kMass = OPS & 1, kDiff = OPS & 2;
    constexpr int NC = kDiff ? (kMass ? 7 : 6) : 1;
    constexpr int NZ = kDiff ? 3 : 1;
    constexpr int Q3 = Q * Q * Q, D3 = D * D * D, QD = Q * D;
    __shared__ double tb[3][QD];           // B^2, BG, G^2 as [a][i]
    __shared__ double sq[NC * Q3];         // D of the element, [t][c][b][a]; then V
    __shared__ double U[NC * Q * Q * D];   // [t][c][b][i]
    static_assert(NZ * Q * D * D <= NC * Q3, "V reuses the storage of D");
    double *V = sq;                        // [z][c][j][i], written once D is no longer read
    const int tid = threadIdx.x;
    for (int t = tid; t < QD; t += kDiagThreads) {
        const double b = tab->B[t], g = tab->G[t];
        tb[T_B2][t] = b * b;
        tb[T_BG][t] = b * g;
        tb[T_G2][t] = g * g;
    }
    const int64_t e = blockIdx.x;
    const double *src = qd + e * (int64_t)(NC * Q3);
    for (int t = tid; t < NC * Q3; t += kDiagThreads) sq[t] = src[t];
    __syncthreads();

    // axis a: U_t(i,b,c) = sum_a X_t[a][i] D_t(a,b,c)
    for (int L = tid; L < NC * Q * Q * D; L += kDiagThreads) {
        const int i = L % D, bc = (L / D) % (Q * Q), t = L / (D * Q * Q);
        int xt = T_B2;  // D_11, D_12, D_22 and the mass term
        if (kDiff && t == 0) xt = T_G2;
        if (kDiff && (t == 1 || t == 2)) xt = T_BG;
        const double *X = tb[xt];
        const double *Dt = sq + t * Q3 + bc * Q;
        double acc = 0.0;
#pragma unroll
        for (int a = 0; a < Q; ++a) acc = fma(X[a * D + i], Dt[a], acc);
        U[L] = acc;
    }
    __syncthreads();

    // axis b: terms grouped by their third-axis table
    for (int L = tid; L < NZ * Q * D * D; L += kDiagThreads) {
        const int i = L % D, j = (L / D) % D, c = (L / (D * D)) % Q, z = L / (D * D * Q);
        auto u = [&](int t, int b) { return U[((t * Q + c) * Q + b) * D + i]; };
        double acc = 0.0;
#pragma unroll
        for (int b = 0; b < Q; ++b) {
            const double b2 = tb[T_B2][b * D + j], bg = tb[T_BG][b * D + j], g2 = tb[T_G2][b * D + j];
            if constexpr (kDiff) {
                if (z == T_B2) {
                    double v = b2 * u(0, b) + 2.0 * bg * u(1, b) + g2 * u(3, b);
                    if constexpr (kMass) v += b2 * u(6, b);
                    acc += v;
                } else if (z == T_BG) {
                    acc += 2.0 * (b2 * u(2, b) + bg * u(4, b));
                } else {
                    acc += b2 * u(5, b);
                }
            } else {
                acc += b2 * u(0, b);
            }
        }
        V[L] = acc;
    }
    __syncthreads();

    // axis c, then the scatter-add through the DOF map
    for (int I = tid; I < D3; I += kDiagThreads) {
        const int i = I % D, j = (I / D) % D, k = I / (D * D);
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < Q; ++c)
#pragma unroll
            for (int z = 0; z < NZ; ++z) acc = fma(tb[z][c * D + k], V[((z * Q + c) * D + j) * D + i], acc);
        unsafeAtomicAdd(diag + emap[e * D3 + I], acc);
    }
}

template <int P>
hipError_t launch_diag_p(const pa_op *op, double *diag, hipStream_t s)
{
    constexpr int D = P + 1;
    const dim3 grid(op->nelem), block(kDiagThreads);
    const int64_t ne = op->nelem;
    if (op->q == P + 1) {
        if (op->ops == 1) hipLaunchKernelGGL((k_diag<D, P + 1, 1>), grid, block, 0, s, ne, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
        if (op->ops == 2) hipLaunchKernelGGL((k_diag<D, P + 1, 2>), grid, block, 0, s, ne, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
        if (op->ops == 3) hipLaunchKernelGGL((k_diag<D, P + 1, 3>), grid, block, 0, s, ne, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
    } else {
        if (op->ops == 1) hipLaunchKernelGGL((k_diag<D, P + 2, 1>), grid, block, 0, s, ne, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
        if (op->ops == 2) hipLaunchKernelGGL((k_diag<D, P + 2, 2>), grid, block, 0, s, ne, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
        if (op->ops == 3) hipLaunchKernelGGL((k_diag<D, P + 2, 3>), grid, block, 0, s, ne, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
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
