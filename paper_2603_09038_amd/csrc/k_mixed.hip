// The paper's own operator: the off-diagonal blocks of the acoustic block operator (eq. (4)),
// pressure p in the continuous order-p space (GLL nodes, DOF map), velocity u in the
// discontinuous order-pu space (Lagrange on pu+1 Gauss-Legendre points per axis, three
// scalar components, element-local), Q Gauss points per axis.  With E_cm = w adj(J)_mc at
// each quadrature point (9 values, the stored D of this operator):
//     yu = G p      : v_c = sum_m E_cm d_m p,      yu_(c,J) = sum_q psi_J v_c
//     yp = -G^T u   : w_m = -sum_c E_cm u_c,        yp_I    = sum_q sum_m d_m phi_I w_m
// One fused kernel computes both with D read once (the paper's fused kernel, Sec. III-G: D
// and D^T applied in the same kernel, the pressure scatter by atomics): per element group
// it gathers p, loads u, runs the sum-factorised forward passes of both spaces, applies D
// and D^T at the quadrature points, and runs the transposed passes, writing yu (element-
// local, plain stores) and scattering yp.  The pressure passes are the diffusion kernel's
// pass descriptors; the velocity passes contract each component with the L2 basis.
#include <hip/hip_runtime.h>

#include "apply_passes.h"
#include "geometry.h"
#include "mixed.h"

namespace hexpa {

namespace {

__device__ __forceinline__ void mx_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

// ------------------------------------------------------------------ velocity passes
// Forward, component CMP, contraction of its fastest index with the L2 basis values
// (A[o][k] = Bu[o][k]); per-component tensors are stored one after the other.
//   VX: U_c[n=(j,k)][i] -> [a][k][j];  VY: [n=(k,a)][j] -> [b][a][k];  VZ: [n=(a,b)][k] -> [c][b][a]
template <int DU, int Q, int CMP, int STAGE>
struct VFwd {
    static constexpr int NIN = STAGE == 0 ? DU * DU * DU : (STAGE == 1 ? Q * DU * DU : Q * Q * DU);
    static constexpr int NCOL = STAGE == 0 ? DU * DU : (STAGE == 1 ? DU * Q : Q * Q);
    static constexpr int C = DU, CS = DU, NT = 1, O = Q;
    static constexpr int OUT = CMP * Q * NCOL, OF = NCOL, OSTR = NCOL;
    __device__ static constexpr int in_off(int) { return CMP * NIN; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, DU); }
};
// Transposed, component CMP: contraction of the fastest (quadrature) index with Bu^T.
//   TX: V_c[n=(b,c)][a] -> [i][c][b];  TY: [n=(c,i)][b] -> [j][i][c];  TZ: [n=(i,j)][c] -> [k][j][i]
template <int DU, int Q, int CMP, int STAGE>
struct VTrn {
    static constexpr int NIN = STAGE == 0 ? Q * Q * Q : (STAGE == 1 ? DU * Q * Q : DU * DU * Q);
    static constexpr int NCOL = STAGE == 0 ? Q * Q : (STAGE == 1 ? Q * DU : DU * DU);
    static constexpr int C = Q, CS = Q, NT = 1, O = DU;
    static constexpr int OUT = CMP * DU * NCOL, OF = NCOL, OSTR = NCOL;
    __device__ static constexpr int in_off(int) { return CMP * NIN; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, DU); }
};

// element-local output of the last velocity pass, yu[e][c][k][j][i]
struct DirectOut {
    double *y;  // the group's first element
    int stride, nv;
    __device__ __forceinline__ void put(int e, int addr, double v) const
    {
        if (e < nv) y[(int64_t)e * stride + addr] = v;
    }
};

template <int DP, int DU, int Q, int NT_ = 128, int BUDGET = kMixLdsBudget / 2>
struct MixShape {
    using S = Shape<DP, Q, 2>;  // the pressure chain: the diffusion kernel's tensors
    static constexpr int NU = DU * DU * DU, Q3 = Q * Q * Q, D3 = DP * DP * DP;
    static constexpr int SZ_A = S::SZ_A, SZ_B = S::SZ_B;
    // velocity ping-pong regions: U (3 NU), VY and TX outputs (3 Q^2 DU) | VX and TY outputs
    // (3 Q DU^2), VZ output (3 Q^3)
    static constexpr int SZ_VA = cmax(3 * NU, 3 * Q * Q * DU) | 1;
    static constexpr int SZ_VB = cmax(3 * Q * DU * DU, 3 * Q3) | 1;
    static constexpr int PER = 8 * (SZ_A + SZ_B + SZ_VA + SZ_VB) + 4 * D3;
    static constexpr int E = cclamp(BUDGET / PER, 1, 16);
    static constexpr int NT = NT_;
    static constexpr int NS = (E * Q3 + NT - 1) / NT;  // quadrature-point slots per thread
};

template <int DP, int DU, int Q>
__global__ __launch_bounds__(128, 3) void k_mixed(int nelem, int ngroups, const int32_t *__restrict__ emap,
                                                  const double *__restrict__ qd, const DevTables *__restrict__ tabp,
                                                  const DevTables *__restrict__ tabu, const double *__restrict__ pv,
                                                  const double *__restrict__ u, double *__restrict__ yu,
                                                  double *__restrict__ yp)
{
    using MS = MixShape<DP, DU, Q>;
    using S = typename MS::S;
    using CH = Chan<Q, false>;
    constexpr int E = MS::E, NT = MS::NT, NS = MS::NS, Q3 = MS::Q3, D3 = MS::D3, NU = MS::NU;
    static_assert(S::DP == DP && S::QP == Q, "the pressure tensors are unpadded at the instantiated orders");
    // the vector-ALU passes read only the columns they own: no tile slack
    __shared__ double bufA[E * MS::SZ_A];
    __shared__ double bufB[E * MS::SZ_B];
    __shared__ double bufVA[E * MS::SZ_VA];
    __shared__ double bufVB[E * MS::SZ_VB];
    __shared__ int32_t lmap[E * D3];
    const int tid = threadIdx.x;
    // Persistent workgroups walking a strided list of element groups.  While group g is
    // contracted, the next group's DOF map, pressure gather and velocity are loaded into
    // registers (after the forward passes), and its D after the D-step.
    constexpr int NMP = (E * D3 + NT - 1) / NT;      // map / pressure slots per thread
    constexpr int NMU = (E * 3 * NU + NT - 1) / NT;  // velocity slots per thread
    auto load_d = [&](int gg, double (&dq)[NS][9]) {
        const int e0 = gg * E, nv = min(E, nelem - e0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int L = tid + s * NT;
            const int e = L / Q3, r = L - e * Q3;
            const bool ok = L < E * Q3 && e < nv;
            const double *src = qd + (int64_t)(e0 + (ok ? e : 0)) * (9 * Q3) + r;
#pragma unroll
            for (int c = 0; c < 9; ++c) dq[s][c] = ok ? __builtin_nontemporal_load(src + c * Q3) : 0.0;
        }
    };
    auto load_map = [&](int gg, int32_t (&mm)[NMP]) {
        const int e0 = gg * E, nv = gg < ngroups ? min(E, nelem - e0) : 0;
#pragma unroll
        for (int s = 0; s < NMP; ++s) {
            const int L = tid + s * NT;
            int e, I;
            row_node<DP, E>(L, e, I);
            mm[s] = (L < E * D3 && e < nv) ? emap[(int64_t)(e0 + e) * D3 + I] : -1;
        }
    };
    auto load_p = [&](const int32_t (&mm)[NMP], double (&pp)[NMP]) {
#pragma unroll
        for (int s = 0; s < NMP; ++s) pp[s] = mm[s] >= 0 ? pv[mm[s]] : 0.0;
    };
    auto load_u = [&](int gg, double (&uu)[NMU]) {
        const int e0 = gg * E, nv = gg < ngroups ? min(E, nelem - e0) : 0;
#pragma unroll
        for (int s = 0; s < NMU; ++s) {
            const int L = tid + s * NT;
            const int e = L / (3 * NU);
            uu[s] = (L < E * 3 * NU && e < nv) ? u[(int64_t)e0 * 3 * NU + L] : 0.0;
        }
    };
    int g = blockIdx.x;
    if (g >= ngroups) return;
    double dq[NS][9], pcur[NMP], ucur[NMU];
    int32_t mcur[NMP];
    load_d(g, dq);
    load_map(g, mcur);
    load_p(mcur, pcur);
    load_u(g, ucur);
    for (;;) {
        const int e0 = g * E, nv = min(E, nelem - e0);
        const int gn = g + gridDim.x;
        const bool more = gn < ngroups;
        // stage the group: the DOF map, the pressure tile (unpadded at these orders, so
        // X[n][i] is the natural node order) and the element-local velocity
#pragma unroll
        for (int s = 0; s < NMP; ++s) {
            const int L = tid + s * NT;
            if (L < E * D3) {
                int e, I;
                row_node<DP, E>(L, e, I);
                lmap[e * D3 + I] = mcur[s];
                bufA[e * MS::SZ_A + I] = pcur[s];
            }
        }
#pragma unroll
        for (int s = 0; s < NMU; ++s) {
            const int L = tid + s * NT;
            if (L < E * 3 * NU) {
                const int e = L / (3 * NU), r = L - e * 3 * NU;
                bufVA[e * MS::SZ_VA + r] = ucur[s];
            }
        }
        int32_t mnext[NMP];
        load_map(gn, mnext);
        mx_barrier();

        // forward passes: the pressure gradient (B and G along each axis) and the velocity
        // values at the quadrature points, three components
        valu_pass<DF1<DP, Q, false>, E, NT>(bufA, MS::SZ_A, tabp, LdsOut<double>{bufB, MS::SZ_B}, tid);
        valu_pass<VFwd<DU, Q, 0, 0>, E, NT>(bufVA, MS::SZ_VA, tabu, LdsOut<double>{bufVB, MS::SZ_VB}, tid);
        valu_pass<VFwd<DU, Q, 1, 0>, E, NT>(bufVA, MS::SZ_VA, tabu, LdsOut<double>{bufVB, MS::SZ_VB}, tid);
        valu_pass<VFwd<DU, Q, 2, 0>, E, NT>(bufVA, MS::SZ_VA, tabu, LdsOut<double>{bufVB, MS::SZ_VB}, tid);
        mx_barrier();
        valu_pass<DF2a<DP, Q, false>, E, NT>(bufB, MS::SZ_B, tabp, LdsOut<double>{bufA, MS::SZ_A}, tid);
        valu_pass<DF2b<DP, Q, false>, E, NT>(bufB, MS::SZ_B, tabp, LdsOut<double>{bufA, MS::SZ_A}, tid);
        valu_pass<VFwd<DU, Q, 0, 1>, E, NT>(bufVB, MS::SZ_VB, tabu, LdsOut<double>{bufVA, MS::SZ_VA}, tid);
        valu_pass<VFwd<DU, Q, 1, 1>, E, NT>(bufVB, MS::SZ_VB, tabu, LdsOut<double>{bufVA, MS::SZ_VA}, tid);
        valu_pass<VFwd<DU, Q, 2, 1>, E, NT>(bufVB, MS::SZ_VB, tabu, LdsOut<double>{bufVA, MS::SZ_VA}, tid);
        mx_barrier();
        valu_pass<DF3a<DP, Q, false>, E, NT>(bufA, MS::SZ_A, tabp, LdsOut<double>{bufB, MS::SZ_B}, tid);
        valu_pass<DF3b<DP, Q, false>, E, NT>(bufA, MS::SZ_A, tabp, LdsOut<double>{bufB, MS::SZ_B}, tid);
        valu_pass<DF3c<DP, Q, false>, E, NT>(bufA, MS::SZ_A, tabp, LdsOut<double>{bufB, MS::SZ_B}, tid);
        valu_pass<VFwd<DU, Q, 0, 2>, E, NT>(bufVA, MS::SZ_VA, tabu, LdsOut<double>{bufVB, MS::SZ_VB}, tid);
        valu_pass<VFwd<DU, Q, 1, 2>, E, NT>(bufVA, MS::SZ_VA, tabu, LdsOut<double>{bufVB, MS::SZ_VB}, tid);
        valu_pass<VFwd<DU, Q, 2, 2>, E, NT>(bufVA, MS::SZ_VA, tabu, LdsOut<double>{bufVB, MS::SZ_VB}, tid);
        double pnext[NMP], unext[NMU];
        load_p(mnext, pnext);  // the next group's map has had the forward passes to arrive
        load_u(gn, unext);
        mx_barrier();

        // D and D^T at the quadrature points: v = E grad_ref p into the velocity channels,
        // w = -E^T u into the pressure-gradient channels
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int L = tid + s * NT;
            if (L < E * Q3) {
                const int e = L / Q3, r = L - e * Q3;
                double *G = bufB + e * MS::SZ_B + CH::qpos(r);
                double *V = bufVB + e * MS::SZ_VB + r;
                const double g0 = G[CH::X], g1 = G[CH::Y], g2 = G[CH::Z];
                const double u0 = V[0], u1 = V[Q3], u2 = V[2 * Q3];
                const double *Em = dq[s];
                V[0] = Em[0] * g0 + Em[1] * g1 + Em[2] * g2;
                V[Q3] = Em[3] * g0 + Em[4] * g1 + Em[5] * g2;
                V[2 * Q3] = Em[6] * g0 + Em[7] * g1 + Em[8] * g2;
                G[CH::X] = -(Em[0] * u0 + Em[3] * u1 + Em[6] * u2);
                G[CH::Y] = -(Em[1] * u0 + Em[4] * u1 + Em[7] * u2);
                G[CH::Z] = -(Em[2] * u0 + Em[5] * u1 + Em[8] * u2);
            }
        }
        if (more) load_d(gn, dq);  // the next group's D, in flight during the transposed passes
        mx_barrier();

        // transposed passes: the gradient-transpose of w into the pressure space (scatter-add),
        // and the velocity test functions against v (element-local stores)
        valu_pass<DT1<DP, Q, false, CH::X, 0, true>, E, NT>(bufB, MS::SZ_B, tabp, LdsOut<double>{bufA, MS::SZ_A}, tid);
        valu_pass<DT1<DP, Q, false, CH::Y, 1, false>, E, NT>(bufB, MS::SZ_B, tabp, LdsOut<double>{bufA, MS::SZ_A}, tid);
        valu_pass<DT1<DP, Q, false, CH::Z, 2, false>, E, NT>(bufB, MS::SZ_B, tabp, LdsOut<double>{bufA, MS::SZ_A}, tid);
        valu_pass<VTrn<DU, Q, 0, 0>, E, NT>(bufVB, MS::SZ_VB, tabu, LdsOut<double>{bufVA, MS::SZ_VA}, tid);
        valu_pass<VTrn<DU, Q, 1, 0>, E, NT>(bufVB, MS::SZ_VB, tabu, LdsOut<double>{bufVA, MS::SZ_VA}, tid);
        valu_pass<VTrn<DU, Q, 2, 0>, E, NT>(bufVB, MS::SZ_VB, tabu, LdsOut<double>{bufVA, MS::SZ_VA}, tid);
        mx_barrier();
        valu_pass<DT2a<DP, Q, false>, E, NT>(bufA, MS::SZ_A, tabp, LdsOut<double>{bufB, MS::SZ_B}, tid);
        valu_pass<DT2b<DP, Q, false>, E, NT>(bufA, MS::SZ_A, tabp, LdsOut<double>{bufB, MS::SZ_B}, tid);
        valu_pass<VTrn<DU, Q, 0, 1>, E, NT>(bufVA, MS::SZ_VA, tabu, LdsOut<double>{bufVB, MS::SZ_VB}, tid);
        valu_pass<VTrn<DU, Q, 1, 1>, E, NT>(bufVA, MS::SZ_VA, tabu, LdsOut<double>{bufVB, MS::SZ_VB}, tid);
        valu_pass<VTrn<DU, Q, 2, 1>, E, NT>(bufVA, MS::SZ_VA, tabu, LdsOut<double>{bufVB, MS::SZ_VB}, tid);
        mx_barrier();
        valu_pass<DT3<DP, Q, false>, E, NT>(bufB, MS::SZ_B, tabp, LdsOut<double>{bufA, MS::SZ_A}, tid);
        const DirectOut dout{yu + (int64_t)e0 * 3 * NU, 3 * NU, nv};
        valu_pass<VTrn<DU, Q, 0, 2>, E, NT>(bufVB, MS::SZ_VB, tabu, dout, tid);
        valu_pass<VTrn<DU, Q, 1, 2>, E, NT>(bufVB, MS::SZ_VB, tabu, dout, tid);
        valu_pass<VTrn<DU, Q, 2, 2>, E, NT>(bufVB, MS::SZ_VB, tabu, dout, tid);
        mx_barrier();
        scatter_group<DP, E, NT, MS::SZ_A, true>(bufA, lmap, yp, tid);
        if (!more) break;
        mx_barrier();  // LDS is rewritten by the next group
        g = gn;
#pragma unroll
        for (int s = 0; s < NMP; ++s) {
            mcur[s] = mnext[s];
            pcur[s] = pnext[s];
        }
#pragma unroll
        for (int s = 0; s < NMU; ++s) ucur[s] = unext[s];
    }
}

// E_cm = w adj(J)_mc at every (element, quadrature point): the rows of adj(J) are the cross
// products of the Jacobian columns.  Layout [e][c][m][Q^3].  Flags det J <= 0.
__global__ void k_mixed_qdata(int64_t nelem, int q, const double *__restrict__ vert, const int32_t *__restrict__ hex,
                              const DevTables *__restrict__ tab, double *__restrict__ qd, int *__restrict__ bad)
{
    const int q3 = q * q * q;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nelem * q3) return;
    const int64_t e = idx / q3;
    const int r = (int)(idx - e * q3);
    const int a = r % q, b = (r / q) % q, c = r / (q * q);
    Hex h;
    load_hex(vert, hex, e, h);
    double x[3], J[3][3];
    map_point(h, tab->x[a], tab->x[b], tab->x[c], x, J);
    const double col0[3] = {J[0][0], J[1][0], J[2][0]};
    const double col1[3] = {J[0][1], J[1][1], J[2][1]};
    const double col2[3] = {J[0][2], J[1][2], J[2][2]};
    double R[3][3];
    cross(col1, col2, R[0]);
    cross(col2, col0, R[1]);
    cross(col0, col1, R[2]);
    const double det = col0[0] * R[0][0] + col0[1] * R[0][1] + col0[2] * R[0][2];
    if (!(det > 0.0)) *bad = 1;
    const double w = tab->w[a] * tab->w[b] * tab->w[c];
    double *out = qd + e * (int64_t)9 * q3 + r;
#pragma unroll
    for (int cc = 0; cc < 3; ++cc)
#pragma unroll
        for (int m = 0; m < 3; ++m) out[(cc * 3 + m) * q3] = w * R[m][cc];
}

// Row-sum lumped masses, one workgroup per element: mu[e][J] = rho sum_q w detJ psi_J and
// mp += sum_q w detJ phi_I / bulk (atomic over the elements sharing a pressure node).
template <int DP, int DU, int Q>
__global__ __launch_bounds__(256) void k_mixed_lumped(int64_t nelem, const double *__restrict__ vert,
                                                      const int32_t *__restrict__ hex, const int32_t *__restrict__ emap,
                                                      const DevTables *__restrict__ tabp,
                                                      const DevTables *__restrict__ tabu, double rho, double bulk,
                                                      double *__restrict__ mu, double *__restrict__ mp)
{
    constexpr int Q3 = Q * Q * Q, NU = DU * DU * DU, D3 = DP * DP * DP;
    __shared__ double wdet[Q3];
    const int64_t e = blockIdx.x;
    Hex h;
    load_hex(vert, hex, e, h);
    for (int r = threadIdx.x; r < Q3; r += blockDim.x) {
        const int a = r % Q, b = (r / Q) % Q, c = r / (Q * Q);
        double x[3], J[3][3];
        map_point(h, tabp->x[a], tabp->x[b], tabp->x[c], x, J);
        const double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) -
                           J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0]) +
                           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        wdet[r] = tabp->w[a] * tabp->w[b] * tabp->w[c] * det;
    }
    __syncthreads();
    for (int J = threadIdx.x; J < NU; J += blockDim.x) {
        const int j1 = J % DU, j2 = (J / DU) % DU, j3 = J / (DU * DU);
        double acc = 0.0;
        for (int r = 0; r < Q3; ++r) {
            const int a = r % Q, b = (r / Q) % Q, c = r / (Q * Q);
            acc += wdet[r] * tB(tabu, a, j1, DU) * tB(tabu, b, j2, DU) * tB(tabu, c, j3, DU);
        }
        mu[e * NU + J] = rho * acc;
    }
    for (int I = threadIdx.x; I < D3; I += blockDim.x) {
        const int i1 = I % DP, i2 = (I / DP) % DP, i3 = I / (DP * DP);
        double acc = 0.0;
        for (int r = 0; r < Q3; ++r) {
            const int a = r % Q, b = (r / Q) % Q, c = r / (Q * Q);
            acc += wdet[r] * tB(tabp, a, i1, DP) * tB(tabp, b, i2, DP) * tB(tabp, c, i3, DP);
        }
        unsafeAtomicAdd(mp + emap[e * D3 + I], acc / bulk);
    }
}

// One RK4 stage combination over a vector: k = -y minv (the stage derivative), then
// acc = k (first stage) or acc + ca k, and either xs = x + cx k (stages 1-3) or, at the last
// stage, x = x + cx (acc + k).
__global__ void k_rk_stage(int64_t n, const double *__restrict__ y, const double *__restrict__ minv, double *__restrict__ x,
                           double *__restrict__ acc, double *__restrict__ xs, int first, double ca, double cx, int last)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double k = -y[i] * minv[i];
        if (last) {
            x[i] = fma(cx, acc[i] + k, x[i]);
        } else {
            acc[i] = first ? k : fma(ca, k, acc[i]);
            xs[i] = fma(cx, k, x[i]);
        }
    }
}

template <int DP, int DU, int Q>
hipError_t launch_mixed_t(const pa_mixed *m, const double *u, const double *p, double *yu, double *yp, hipStream_t s)
{
    using MS = MixShape<DP, DU, Q>;
    const int ngroups = (m->nelem + MS::E - 1) / MS::E;
    if (ngroups == 0) return hipSuccess;
    static int cap = 0;
    if (cap == 0) {
        int per_cu = 0, dev = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_mixed<DP, DU, Q>, MS::NT, 0) != hipSuccess || per_cu < 1)
            per_cu = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
            ncu = 256;
        cap = per_cu * ncu;
    }
    int nb = ngroups < cap ? ngroups : cap;
    if (m->grid_cap > 0 && m->grid_cap < nb) nb = m->grid_cap;
    hipLaunchKernelGGL((k_mixed<DP, DU, Q>), dim3(nb), dim3(MS::NT), 0, s, m->nelem, ngroups, m->d_emap, m->d_qdata,
                       m->d_tabp, m->d_tabu, p, u, yu, yp);
    return hipGetLastError();
}

template <int DP, int DU, int Q>
hipError_t launch_mixed_lumped_t(const pa_mixed *m, double *mu, double *mp, hipStream_t s)
{
    hipLaunchKernelGGL((k_mixed_lumped<DP, DU, Q>), dim3(m->nelem), dim3(256), 0, s, (int64_t)m->nelem, m->d_vert,
                       m->d_hex, m->d_emap, m->d_tabp, m->d_tabu, m->rho, m->bulk, mu, mp);
    return hipGetLastError();
}

}  // namespace

bool mixed_supported(int p, int pu, int q) { return (p == 4 && pu == 3 && q == 5) || (p == 2 && pu == 1 && q == 3); }

int mixed_elems_per_group(int p, int pu, int q)
{
    if (p == 4 && pu == 3 && q == 5) return MixShape<5, 4, 5>::E;
    if (p == 2 && pu == 1 && q == 3) return MixShape<3, 2, 3>::E;
    return 0;
}

hipError_t launch_mixed(const pa_mixed *m, const double *u, const double *p, double *yu, double *yp, hipStream_t s)
{
    if (m->p == 4) return launch_mixed_t<5, 4, 5>(m, u, p, yu, yp, s);
    return launch_mixed_t<3, 2, 3>(m, u, p, yu, yp, s);
}

hipError_t launch_mixed_qdata(const pa_mixed *m, int *bad, hipStream_t s)
{
    const int64_t n = (int64_t)m->nelem * m->q * m->q * m->q;
    hipLaunchKernelGGL(k_mixed_qdata, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, (int64_t)m->nelem, m->q,
                       m->d_vert, m->d_hex, m->d_tabp, m->d_qdata, bad);
    return hipGetLastError();
}

hipError_t launch_mixed_lumped(const pa_mixed *m, double *mu, double *mp, hipStream_t s)
{
    if (m->p == 4) return launch_mixed_lumped_t<5, 4, 5>(m, mu, mp, s);
    return launch_mixed_lumped_t<3, 2, 3>(m, mu, mp, s);
}

hipError_t launch_rk_stage(int64_t n, const double *y, const double *minv, double *x, double *acc, double *xs,
                           int first, double ca, double cx, int last, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_rk_stage, dim3((unsigned)(nb < 8192 ? nb : 8192)), dim3(256), 0, s, n, y, minv, x, acc, xs,
                       first, ca, cx, last);
    return hipGetLastError();
}

}  // namespace hexpa
