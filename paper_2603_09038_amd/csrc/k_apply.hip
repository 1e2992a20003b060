// Fused PA apply kernels (mass, diffusion, mass+diffusion) and their launcher.
#include "apply_passes.h"

namespace hexpa {

// Element-group index of this workgroup.  Workgroups are dealt to the 8 XCDs round-robin
// (block b runs on XCD b % 8); remapping gives every XCD one contiguous range of element
// groups, so neighbouring elements (which share DOFs of x and y) meet in the same L2.
__device__ __forceinline__ int xcd_group(int b, int ngroups)
{
    const int per = ngroups >> 3, rem = ngroups & 7;
    const int x = b & 7, i = b >> 3;
    return x * per + (x < rem ? x : rem) + i;
}

template <int D, int Q, int OPS, bool MFMA, bool ATOMIC>
__global__ __launch_bounds__(kThreads) void k_apply(int nelem, int ngroups, const int32_t *__restrict__ elist,
                                                    const int32_t *__restrict__ emap,
                                                    const double *__restrict__ qd,
                                                    const DevTables *__restrict__ tab,
                                                    const double *__restrict__ x, double *__restrict__ y)
{
    using S = Shape<D, Q, OPS>;
    constexpr int E = S::E, D3 = S::D3, Q3 = S::Q3, NS = S::NS, NC = S::NCOMP;
    constexpr bool M = S::kMass;
    __shared__ double bufA[E * S::SZ_A];
    __shared__ double bufB[E * S::SZ_B];
    __shared__ int32_t lmap[E * D3];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int g = xcd_group(blockIdx.x, ngroups);
    const int e0 = g * E;
    const int nv = min(E, nelem - e0);

    // Quadrature data of the group, issued first so its HBM latency hides under the
    // forward contractions: slot s of thread tid is qp entry L = tid + s*256 of the group.
    double dq[NS][NC];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int L = tid + s * kThreads;
        const int e = L / Q3, r = L - e * Q3;
        const bool ok = e < nv;
        const int64_t ge = ok ? (elist ? elist[e0 + e] : e0 + e) : 0;
        const double *src = qd + ge * (int64_t)(NC * Q3) + r;
#pragma unroll
        for (int c = 0; c < NC; ++c) dq[s][c] = ok ? __builtin_nontemporal_load(src + c * Q3) : 0.0;
    }

    // Gather x_E = G_e x into X[e][n=(j,k)][i] (= local node order) and keep the map.
    for (int L = tid; L < E * D3; L += kThreads) {
        const int e = L / D3, I = L - e * D3;
        int32_t gi = -1;
        double v = 0.0;
        if (e < nv) {
            const int64_t ge = elist ? elist[e0 + e] : e0 + e;
            gi = emap[ge * D3 + I];
            v = x[gi];
        }
        lmap[L] = gi;
        bufA[e * S::SZ_A + I] = v;
    }

    constexpr int RBF = (S::kDiff ? (2 * Q + 15) / 16 : (Q + 15) / 16);
    __syncthreads();

    if constexpr (S::kDiff) {
        using F1 = DF1<D, Q, M>; using F2 = DF2<D, Q, M>; using F3 = DF3<D, Q, M>;
        using T1a = DT1a<D, Q, M>; using T1b = DT1b<D, Q, M>;
        using T2a = DT2a<D, Q, M>; using T2b = DT2b<D, Q, M>; using T3 = DT3<D, Q, M>;
        if constexpr (MFMA) {
            double aF[PassRegs<F1>::RB][PassRegs<F1>::KC];
            load_a<F1>(tab, aF, lane);
            mfma_pass<F1, E>(bufA, S::SZ_A, aF, LdsOut{bufB, S::SZ_B}, wave, lane);
            __syncthreads();
            mfma_pass<F2, E>(bufB, S::SZ_B, aF, LdsOut{bufA, S::SZ_A}, wave, lane);
            __syncthreads();
            mfma_pass<F3, E>(bufA, S::SZ_A, aF, LdsOut{bufB, S::SZ_B}, wave, lane);
        } else {
            valu_pass<F1, E>(bufA, S::SZ_A, tab, LdsOut{bufB, S::SZ_B}, tid);
            __syncthreads();
            valu_pass<F2, E>(bufB, S::SZ_B, tab, LdsOut{bufA, S::SZ_A}, tid);
            __syncthreads();
            valu_pass<F3, E>(bufA, S::SZ_A, tab, LdsOut{bufB, S::SZ_B}, tid);
        }
        __syncthreads();
        // D at quadrature points: v = D grad_ref u (symmetric 3x3), v_u = D_m u.
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int L = tid + s * kThreads;
            if (L < E * Q3) {
                const int e = L / Q3, r = L - e * Q3;
                double *V = bufB + e * S::SZ_B + r;
                const double g0 = V[0], g1 = V[Q3], g2 = V[2 * Q3];
                const double *Dm = dq[s];
                V[0] = Dm[0] * g0 + Dm[1] * g1 + Dm[2] * g2;
                V[Q3] = Dm[1] * g0 + Dm[3] * g1 + Dm[4] * g2;
                V[2 * Q3] = Dm[2] * g0 + Dm[4] * g1 + Dm[5] * g2;
                if constexpr (M) V[3 * Q3] = Dm[6] * V[3 * Q3];
            }
        }
        __syncthreads();
        if constexpr (MFMA) {
            double aTG[PassRegs<T1a>::RB][PassRegs<T1a>::KC];
            double aTB[PassRegs<T1b>::RB][PassRegs<T1b>::KC];
            load_a<T1a>(tab, aTG, lane);
            load_a<T1b>(tab, aTB, lane);
            mfma_pass<T1a, E>(bufB, S::SZ_B, aTG, LdsOut{bufA, S::SZ_A}, wave, lane);
            mfma_pass<T1b, E>(bufB, S::SZ_B, aTB, LdsOut{bufA, S::SZ_A}, wave, lane);
            __syncthreads();
            double a2[PassRegs<T2a>::RB][PassRegs<T2a>::KC];
            load_a<T2a>(tab, a2, lane);
            mfma_pass<T2a, E>(bufA, S::SZ_A, a2, LdsOut{bufB, S::SZ_B}, wave, lane);
            mfma_pass<T2b, E>(bufA, S::SZ_A, aTB, LdsOut{bufB, S::SZ_B}, wave, lane);
            __syncthreads();
            double a3[PassRegs<T3>::RB][PassRegs<T3>::KC];
            load_a<T3>(tab, a3, lane);
            mfma_pass<T3, E>(bufB, S::SZ_B, a3, GlobalOut<ATOMIC>{y, lmap, D3}, wave, lane);
        } else {
            valu_pass<T1a, E>(bufB, S::SZ_B, tab, LdsOut{bufA, S::SZ_A}, tid);
            valu_pass<T1b, E>(bufB, S::SZ_B, tab, LdsOut{bufA, S::SZ_A}, tid);
            __syncthreads();
            valu_pass<T2a, E>(bufA, S::SZ_A, tab, LdsOut{bufB, S::SZ_B}, tid);
            valu_pass<T2b, E>(bufA, S::SZ_A, tab, LdsOut{bufB, S::SZ_B}, tid);
            __syncthreads();
            valu_pass<T3, E>(bufB, S::SZ_B, tab, GlobalOut<ATOMIC>{y, lmap, D3}, tid);
        }
    } else {
        using F1 = MF1<D, Q>; using F2 = MF2<D, Q>; using F3 = MF3<D, Q>;
        using T1 = MT1<D, Q>; using T2 = MT2<D, Q>; using T3 = MT3<D, Q>;
        if constexpr (MFMA) {
            double aF[PassRegs<F1>::RB][PassRegs<F1>::KC];
            load_a<F1>(tab, aF, lane);
            mfma_pass<F1, E>(bufA, S::SZ_A, aF, LdsOut{bufB, S::SZ_B}, wave, lane);
            __syncthreads();
            mfma_pass<F2, E>(bufB, S::SZ_B, aF, LdsOut{bufA, S::SZ_A}, wave, lane);
            __syncthreads();
            mfma_pass<F3, E>(bufA, S::SZ_A, aF, LdsOut{bufB, S::SZ_B}, wave, lane);
        } else {
            valu_pass<F1, E>(bufA, S::SZ_A, tab, LdsOut{bufB, S::SZ_B}, tid);
            __syncthreads();
            valu_pass<F2, E>(bufB, S::SZ_B, tab, LdsOut{bufA, S::SZ_A}, tid);
            __syncthreads();
            valu_pass<F3, E>(bufA, S::SZ_A, tab, LdsOut{bufB, S::SZ_B}, tid);
        }
        __syncthreads();
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int L = tid + s * kThreads;
            if (L < E * Q3) {
                const int e = L / Q3, r = L - e * Q3;
                bufB[e * S::SZ_B + r] *= dq[s][0];
            }
        }
        __syncthreads();
        if constexpr (MFMA) {
            double aT[PassRegs<T1>::RB][PassRegs<T1>::KC];
            load_a<T1>(tab, aT, lane);
            mfma_pass<T1, E>(bufB, S::SZ_B, aT, LdsOut{bufA, S::SZ_A}, wave, lane);
            __syncthreads();
            mfma_pass<T2, E>(bufA, S::SZ_A, aT, LdsOut{bufB, S::SZ_B}, wave, lane);
            __syncthreads();
            mfma_pass<T3, E>(bufB, S::SZ_B, aT, GlobalOut<ATOMIC>{y, lmap, D3}, wave, lane);
        } else {
            valu_pass<T1, E>(bufB, S::SZ_B, tab, LdsOut{bufA, S::SZ_A}, tid);
            __syncthreads();
            valu_pass<T2, E>(bufA, S::SZ_A, tab, LdsOut{bufB, S::SZ_B}, tid);
            __syncthreads();
            valu_pass<T3, E>(bufB, S::SZ_B, tab, GlobalOut<ATOMIC>{y, lmap, D3}, tid);
        }
    }
    (void)RBF;
}

// ------------------------------------------------------------------ launcher
template <int D, int Q, int OPS>
static hipError_t launch_t(const pa_op *op, int variant, const double *x, double *y, const int32_t *elist, int n,
                           hipStream_t s)
{
    using S = Shape<D, Q, OPS>;
    const int ngroups = (n + S::E - 1) / S::E;
    if (ngroups == 0) return hipSuccess;
    dim3 grid(ngroups), block(kThreads);
    switch (variant) {
    case PA_VARIANT_VALU:
        hipLaunchKernelGGL((k_apply<D, Q, OPS, false, true>), grid, block, 0, s, n, ngroups, elist, op->d_elem_dofs,
                           op->d_qdata, op->d_tab, x, y);
        break;
    case PA_VARIANT_MFMA_COLORED:
        hipLaunchKernelGGL((k_apply<D, Q, OPS, true, false>), grid, block, 0, s, n, ngroups, elist, op->d_elem_dofs,
                           op->d_qdata, op->d_tab, x, y);
        break;
    default:
        hipLaunchKernelGGL((k_apply<D, Q, OPS, true, true>), grid, block, 0, s, n, ngroups, elist, op->d_elem_dofs,
                           op->d_qdata, op->d_tab, x, y);
    }
    return hipGetLastError();
}

template <int P>
static hipError_t launch_p(const pa_op *op, int variant, const double *x, double *y, const int32_t *elist, int n,
                           hipStream_t s, bool *ok)
{
    constexpr int D = P + 1;
    *ok = true;
    if (op->q == P + 1) {
        switch (op->ops) {
        case 1: return launch_t<D, P + 1, 1>(op, variant, x, y, elist, n, s);
        case 2: return launch_t<D, P + 1, 2>(op, variant, x, y, elist, n, s);
        case 3: return launch_t<D, P + 1, 3>(op, variant, x, y, elist, n, s);
        }
    } else if (op->q == P + 2) {
        switch (op->ops) {
        case 1: return launch_t<D, P + 2, 1>(op, variant, x, y, elist, n, s);
        case 2: return launch_t<D, P + 2, 2>(op, variant, x, y, elist, n, s);
        case 3: return launch_t<D, P + 2, 3>(op, variant, x, y, elist, n, s);
        }
    }
    *ok = false;
    return hipSuccess;
}

#ifndef HEXPA_APPLY_P
#error "compile k_apply.hip once per order with -DHEXPA_APPLY_P=<p>"
#endif

#define HEXPA_CAT2(a, b) a##b
#define HEXPA_CAT(a, b) HEXPA_CAT2(a, b)
hipError_t HEXPA_CAT(launch_apply_p, HEXPA_APPLY_P)(const pa_op *op, int variant, const double *x, double *y,
                                                   const int32_t *elist, int n, hipStream_t s, bool *ok)
{
    return launch_p<HEXPA_APPLY_P>(op, variant, x, y, elist, n, s, ok);
}

}  // namespace hexpa
