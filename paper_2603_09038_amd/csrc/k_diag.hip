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

constexpr int kDiagThreads = 256;

// per-axis table index of each stored component (D order 00, 01, 02, 11, 12, 22, mass)
enum : int { T_B2 = 0, T_BG = 1, T_G2 = 2 };

// NR = NC Q^2 contiguous a-rows of D per element; a workgroup takes EPB consecutive
// elements (one at high order, up to 16 at low order so that its threads have work).  The
// first contraction reads D straight from HBM into registers (each thread one a-row), so
// the only LDS arrays are the two intermediate tensors and the tables (about 31 KB at
// Q = 8): several workgroups share a CU and their D streams overlap one another's
// arithmetic.
template <int D, int Q, int OPS>
struct DiagShape {
    static constexpr bool kMass = OPS & 1, kDiff = OPS & 2;
    static constexpr int NC = kDiff ? (kMass ? 7 : 6) : 1;
    static constexpr int NZ = kDiff ? 3 : 1;
    static constexpr int NR = NC * Q * Q;
    static constexpr int EPB = NR >= kDiagThreads ? 1 : (kDiagThreads / NR > 16 ? 16 : kDiagThreads / NR);
};

template <int D, int Q, int OPS>
__global__ __launch_bounds__(kDiagThreads) void k_diag(int64_t nelem, const int32_t *__restrict__ emap,
                                                       const double *__restrict__ qd,
                                                       const DevTables *__restrict__ tab, double *__restrict__ diag)
{
    using S = DiagShape<D, Q, OPS>;
    constexpr bool kMass = S::kMass, kDiff = S::kDiff;
    constexpr int NC = S::NC, NZ = S::NZ, NR = S::NR, EPB = S::EPB;
    constexpr int Q3 = Q * Q * Q, D3 = D * D * D, QD = Q * D;
    constexpr int DP = D | 1;              // odd row pitch of U: the a-row writes spread over the banks
    constexpr int SU = NR * DP, SV = NZ * Q * D * D;
    __shared__ double tb[3][QD];           // B^2, BG, G^2 as [a][i]
    __shared__ double U[EPB * SU];         // per element [t][c][b][i]
    __shared__ double V[EPB * SV];         // per element [z][c][j][i]
    const int tid = threadIdx.x;
    for (int t = tid; t < QD; t += kDiagThreads) {
        const double b = tab->B[t], g = tab->G[t];
        tb[T_B2][t] = b * b;
        tb[T_BG][t] = b * g;
        tb[T_G2][t] = g * g;
    }
    const int64_t e0 = (int64_t)blockIdx.x * EPB;
    const int ne = (int)(nelem - e0 < EPB ? nelem - e0 : EPB);
    const double *src = qd + e0 * (int64_t)(NC * Q3);  // the ne elements' rows are consecutive
    __syncthreads();

    // axis a: U_t(i,b,c) = sum_a X_t[a][i] D_t(a,b,c); row (t,c,b) of D is contiguous in a
    for (int R = tid; R < ne * NR; R += kDiagThreads) {
        const int t = (R % NR) / (Q * Q);
        double d[Q];
#pragma unroll
        for (int a = 0; a < Q; ++a) d[a] = __builtin_nontemporal_load(src + (int64_t)R * Q + a);
        int xt = T_B2;  // D_11, D_12, D_22 and the mass term
        if (kDiff && t == 0) xt = T_G2;
        if (kDiff && (t == 1 || t == 2)) xt = T_BG;
        const double *X = tb[xt];
#pragma unroll
        for (int i = 0; i < D; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int a = 0; a < Q; ++a) acc = fma(X[a * D + i], d[a], acc);
            U[R * DP + i] = acc;
        }
    }
    __syncthreads();

    // axis b: terms grouped by their third-axis table
    for (int L = tid; L < ne * SV; L += kDiagThreads) {
        const int le = L / SV, l = L - le * SV;
        const int i = l % D, j = (l / D) % D, c = (l / (D * D)) % Q, z = l / (D * D * Q);
        const double *Ue = U + le * SU;
        auto u = [&](int t, int b) { return Ue[((t * Q + c) * Q + b) * DP + i]; };
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
    for (int L = tid; L < ne * D3; L += kDiagThreads) {
        const int le = L / D3, I = L - le * D3;
        const int i = I % D, j = (I / D) % D, k = I / (D * D);
        const double *Ve = V + le * SV;
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < Q; ++c)
#pragma unroll
            for (int z = 0; z < NZ; ++z) acc = fma(tb[z][c * D + k], Ve[((z * Q + c) * D + j) * D + i], acc);
        unsafeAtomicAdd(diag + emap[e0 * D3 + L], acc);
    }
}

template <int D, int Q, int OPS>
void launch_diag_k(const pa_op *op, double *diag, hipStream_t s)
{
    constexpr int EPB = DiagShape<D, Q, OPS>::EPB;
    const int64_t ne = op->nelem;
    const dim3 grid((unsigned)((ne + EPB - 1) / EPB)), block(kDiagThreads);
    hipLaunchKernelGGL((k_diag<D, Q, OPS>), grid, block, 0, s, ne, op->d_elem_dofs, op->d_qdata, op->d_tab, diag);
}

template <int D, int Q>
hipError_t launch_diag_q(const pa_op *op, double *diag, hipStream_t s)
{
    if (op->ops == 1) launch_diag_k<D, Q, 1>(op, diag, s);
    if (op->ops == 2) launch_diag_k<D, Q, 2>(op, diag, s);
    if (op->ops == 3) launch_diag_k<D, Q, 3>(op, diag, s);
    return hipGetLastError();
}

template <int P>
hipError_t launch_diag_p(const pa_op *op, double *diag, hipStream_t s)
{
    if (op->q == P + 1) return launch_diag_q<P + 1, P + 1>(op, diag, s);
    return launch_diag_q<P + 1, P + 2>(op, diag, s);
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
