// Fused PA apply kernels (mass, diffusion, mass+diffusion) and their launchers.
//
// One kernel template serves every precision: FP64 with MFMA (v_mfma_f64_4x4x4f64) or
// vector-ALU contractions, and the mixed-precision inner apply (FP32 vectors, FP32 D and
// LDS tensors, FP16/BF16 MFMA contractions with FP32 accumulation).
//
// Persistent workgroups: the grid holds about as many workgroups as the chip keeps
// resident, and each one walks a strided list of element groups.  While group g is being
// contracted, the DOF map and then the gathered x of the group it does next are already
// in flight, so the gather latency overlaps the LDS/MFMA work of the current group.
#include <type_traits>

#include "apply_passes.h"

#ifndef HEXPA_PREFETCH_D
#define HEXPA_PREFETCH_D 0
#endif
#ifndef HEXPA_OVERSUB
#define HEXPA_OVERSUB 1
#endif
#ifndef HEXPA_LATE_D
#define HEXPA_LATE_D 1
#endif
#ifndef HEXPA_MIN_BLOCKS
#define HEXPA_MIN_BLOCKS 3
#endif

namespace hexpa {

constexpr bool kPrefetchD = HEXPA_PREFETCH_D != 0;  // double-buffer D in registers across groups
constexpr bool kLateD = HEXPA_LATE_D != 0;          // load D at the D-step (no prefetch)
constexpr int kOversub = HEXPA_OVERSUB;             // resident-workgroup multiples in the grid (0: one group each)
constexpr int kMinWavesPerEU = HEXPA_MIN_BLOCKS;    // register budget: waves resident per SIMD

// Contraction executors.
enum : int { EX_MFMA64 = 0, EX_VALU64 = 1, EX_MFMA16F = 2, EX_MFMA16B = 3 };
template <int EX>
struct ExT {
    using T = typename std::conditional<(EX >= EX_MFMA16F), float, double>::type;
};

template <class S>
struct GroupRegs {
    static constexpr int NM = (S::E * S::D3 + kThreads - 1) / kThreads;  // map/x slots per thread
};

// D of one group into registers: slot s of thread tid is qp entry L = tid + s*kThreads.
template <class S, class T>
__device__ __forceinline__ void load_qdata(T (&dq)[S::NS][S::NCOMP], const T *__restrict__ qd,
                                           const int32_t *__restrict__ elist, int e0, int nv, int tid)
{
#pragma unroll
    for (int s = 0; s < S::NS; ++s) {
        const int L = tid + s * kThreads;
        const int e = L / S::Q3, r = L - e * S::Q3;
        const bool ok = e < nv;
        const int64_t ge = ok ? (elist ? elist[e0 + e] : e0 + e) : 0;
        const T *src = qd + ge * (int64_t)(S::NCOMP * S::Q3) + r;
#pragma unroll
        for (int c = 0; c < S::NCOMP; ++c) dq[s][c] = ok ? __builtin_nontemporal_load(src + c * S::Q3) : T(0);
    }
}

template <class S>
__device__ __forceinline__ void load_map(int32_t (&m)[GroupRegs<S>::NM], const int32_t *__restrict__ emap,
                                         const int32_t *__restrict__ elist, int e0, int nv, int tid)
{
#pragma unroll
    for (int s = 0; s < GroupRegs<S>::NM; ++s) {
        const int L = tid + s * kThreads;
        const int e = L / S::D3, I = L - e * S::D3;
        int32_t gi = -1;
        if (e < nv) {
            const int64_t ge = elist ? elist[e0 + e] : e0 + e;
            gi = emap[ge * S::D3 + I];
        }
        m[s] = gi;
    }
}

template <class S, class T>
__device__ __forceinline__ void load_x(T (&xv)[GroupRegs<S>::NM], const int32_t (&m)[GroupRegs<S>::NM],
                                       const T *__restrict__ x)
{
#pragma unroll
    for (int s = 0; s < GroupRegs<S>::NM; ++s) xv[s] = m[s] >= 0 ? x[m[s]] : T(0);
}

// One contraction pass with the chosen executor.  MFMA A-operands are read from the LDS
// copy of the tables right before the pass (short live ranges, no hoisting across the
// barriers); the VALU executor reads the tables with uniform loads from global memory.
template <class P, int E, int EX, class T, class Out>
__device__ __forceinline__ void run_pass(const T *in, int szin, const DevTables *stab, const DevTables *gtab,
                                         const Out &out, int tid)
{
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    if constexpr (EX == EX_MFMA64) {
        double a[PassRegs<P>::RT][PassRegs<P>::KC];
        load_a<P>(stab, a, lane);
        mfma_pass<P, E>(in, szin, a, out, wave, lane);
    } else if constexpr (EX == EX_VALU64) {
        valu_pass<P, E>(in, szin, gtab, out, tid);
    } else {
        constexpr bool BF = EX == EX_MFMA16B;
        typename Mfma16<BF>::V a[PassRegs16<P>::RB][PassRegs16<P>::KC];
        load_a16<P, BF>(stab, a, lane);
        mfma16_pass<P, E, BF>(in, szin, a, out, wave, lane);
    }
}

template <int D, int Q, int OPS, int EX, bool ATOMIC>
__global__ __launch_bounds__(kThreads, kMinWavesPerEU) void k_apply(
    int nelem, int ngroups, const int32_t *__restrict__ elist, const int32_t *__restrict__ emap,
    const typename ExT<EX>::T *__restrict__ qd, const DevTables *__restrict__ tab,
    const typename ExT<EX>::T *__restrict__ x, typename ExT<EX>::T *__restrict__ y)
{
    using T = typename ExT<EX>::T;
    using S = Shape<D, Q, OPS, (int)sizeof(T)>;
    constexpr int E = S::E, D3 = S::D3, Q3 = S::Q3, NS = S::NS, NC = S::NCOMP, NM = GroupRegs<S>::NM;
    constexpr bool M = S::kMass;
    __shared__ T bufA[E * S::SZ_A + S::SLACK];
    __shared__ T bufB[E * S::SZ_B + S::SLACK];
    __shared__ int32_t lmap[E * D3];
    __shared__ DevTables stab;  // 1-D tables in LDS: MFMA A-operands are re-read per pass

    const int tid = threadIdx.x;
    for (int i = tid; i < (int)(sizeof(DevTables) / sizeof(double)); i += kThreads)
        reinterpret_cast<double *>(&stab)[i] = reinterpret_cast<const double *>(tab)[i];

    // Workgroup b runs on XCD b % 8.  XCD x owns the contiguous group range
    // [G x / 8, G (x+1) / 8) so neighbouring elements (sharing DOFs of x and y) meet in the
    // same L2; its workgroups take that range's groups round-robin.
    // (Grids of fewer than 8 workgroups just stride over all groups.)
    const int nb = gridDim.x;
    int g, gend, nbx;
    if (nb >= 8) {
        const int xcd = blockIdx.x & 7, slot = blockIdx.x >> 3;
        nbx = (nb >> 3) + (xcd < (nb & 7) ? 1 : 0);
        gend = (int)(((int64_t)ngroups * (xcd + 1)) >> 3);
        g = (int)(((int64_t)ngroups * xcd) >> 3) + slot;
    } else {
        nbx = nb;
        gend = ngroups;
        g = blockIdx.x;
    }
    if (g >= gend) return;

    T dq[NS][NC];
    int32_t mcur[NM];
    T xcur[NM];
    {
        const int e0 = g * E, nv = min(E, nelem - e0);
        if constexpr (!kLateD) load_qdata<S>(dq, qd, elist, e0, nv, tid);
        load_map<S>(mcur, emap, elist, e0, nv, tid);
        load_x<S>(xcur, mcur, x);
    }

    for (;;) {
        const int e0 = g * E, nv = min(E, nelem - e0);
        const int gn = g + nbx;
        const bool more = gn < gend;
        const int e0n = gn * E, nvn = more ? min(E, nelem - e0n) : 0;

        // stage x_E = G_e x (local node order = X[e][n=(j,k)][i]) and the map
#pragma unroll
        for (int s = 0; s < NM; ++s) {
            const int L = tid + s * kThreads;
            if (L < E * D3) {
                const int e = L / D3, I = L - e * D3;
                lmap[L] = mcur[s];
                bufA[e * S::SZ_A + I] = xcur[s];
            }
        }
        int32_t mnext[NM];
        load_map<S>(mnext, emap, elist, e0n, nvn, tid);
        T dnext[kPrefetchD ? NS : 1][NC];
        if constexpr (kPrefetchD) load_qdata<S>(dnext, qd, elist, e0n, nvn, tid);
        __syncthreads();

        // forward contractions
        if constexpr (S::kDiff) {
            run_pass<DF1<D, Q, M>, E, EX>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid);
            __syncthreads();
            run_pass<DF2a<D, Q, M>, E, EX>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid);
            run_pass<DF2b<D, Q, M>, E, EX>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid);
            __syncthreads();
            run_pass<DF3a<D, Q, M>, E, EX>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid);
            run_pass<DF3b<D, Q, M>, E, EX>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid);
            run_pass<DF3c<D, Q, M>, E, EX>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid);
        } else {
            run_pass<MF1<D, Q>, E, EX>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid);
            __syncthreads();
            run_pass<MF2<D, Q>, E, EX>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid);
            __syncthreads();
            run_pass<MF3<D, Q>, E, EX>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid);
        }
        // the next group's map has had the forward passes to arrive: start its x gather
        T xnext[NM];
        load_x<S>(xnext, mnext, x);
        __syncthreads();

        // D at quadrature points: v = D grad_ref u (symmetric 3x3) and/or v_u = D_m u
        if constexpr (kLateD) load_qdata<S>(dq, qd, elist, e0, nv, tid);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int L = tid + s * kThreads;
            if (L < E * Q3) {
                const int e = L / Q3, r = L - e * Q3;
                T *V = bufB + e * S::SZ_B + r;
                const T *Dm = dq[s];
                if constexpr (S::kDiff) {
                    using CH = Chan<Q, M>;
                    const T g0 = V[CH::X], g1 = V[CH::Y], g2 = V[CH::Z];
                    V[CH::X] = Dm[0] * g0 + Dm[1] * g1 + Dm[2] * g2;
                    V[CH::Y] = Dm[1] * g0 + Dm[3] * g1 + Dm[4] * g2;
                    V[CH::Z] = Dm[2] * g0 + Dm[4] * g1 + Dm[5] * g2;
                    if constexpr (M) V[CH::V] = Dm[6] * V[CH::V];
                } else {
                    V[0] *= Dm[0];
                }
            }
        }
        if (more && !kLateD) {
            if constexpr (kPrefetchD) {
#pragma unroll
                for (int s = 0; s < NS; ++s)
#pragma unroll
                    for (int c = 0; c < NC; ++c) dq[s][c] = dnext[s][c];
            } else {
                load_qdata<S>(dq, qd, elist, e0n, nvn, tid);
            }
        }
        __syncthreads();

        // transposed contractions and scatter-add
        if constexpr (S::kDiff) {
            using CH = Chan<Q, M>;
            run_pass<DT1<D, Q, M, CH::X, 0, true>, E, EX>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid);
            run_pass<DT1<D, Q, M, CH::Y, 1, false>, E, EX>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid);
            run_pass<DT1<D, Q, M, CH::Z, 2, false>, E, EX>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid);
            if constexpr (M)
                run_pass<DT1<D, Q, M, CH::V, 3, false>, E, EX>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A},
                                                                tid);
            __syncthreads();
            run_pass<DT2a<D, Q, M>, E, EX>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid);
            run_pass<DT2b<D, Q, M>, E, EX>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid);
            __syncthreads();
            run_pass<DT3<D, Q, M>, E, EX>(bufB, S::SZ_B, &stab, tab, GlobalOut<ATOMIC, T>{y, lmap, D3}, tid);
        } else {
            run_pass<MT1<D, Q>, E, EX>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid);
            __syncthreads();
            run_pass<MT2<D, Q>, E, EX>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid);
            __syncthreads();
            run_pass<MT3<D, Q>, E, EX>(bufB, S::SZ_B, &stab, tab, GlobalOut<ATOMIC, T>{y, lmap, D3}, tid);
        }
        if (!more) break;
        __syncthreads();  // LDS (X, map) is rewritten by the next group
        g = gn;
#pragma unroll
        for (int s = 0; s < NM; ++s) {
            mcur[s] = mnext[s];
            xcur[s] = xnext[s];
        }
    }
}

// ------------------------------------------------------------------ launchers
template <int D, int Q, int OPS, int EX, bool ATOMIC>
static hipError_t launch_k(const pa_op *op, const typename ExT<EX>::T *qd, const typename ExT<EX>::T *x,
                           typename ExT<EX>::T *y, const int32_t *elist, int n, hipStream_t s)
{
    using S = Shape<D, Q, OPS, (int)sizeof(typename ExT<EX>::T)>;
    const int ngroups = (n + S::E - 1) / S::E;
    if (ngroups == 0) return hipSuccess;
    auto kern = k_apply<D, Q, OPS, EX, ATOMIC>;
    int nblocks = ngroups;
    if (kOversub > 0) {
        // resident capacity of the device for this kernel (queried once)
        static int cap = 0;
        if (cap == 0) {
            int per_cu = 0, dev = 0, ncu = 0;
            if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kThreads, 0) != hipSuccess || per_cu < 1)
                per_cu = 1;
            if (hipGetDevice(&dev) != hipSuccess ||
                hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
                ncu = 256;
            cap = per_cu * ncu * kOversub;
        }
        nblocks = ngroups < cap ? ngroups : cap;
    }
    hipLaunchKernelGGL(kern, dim3(nblocks), dim3(kThreads), 0, s, n, ngroups, elist, op->d_elem_dofs, qd, op->d_tab,
                       x, y);
    return hipGetLastError();
}

template <int D, int Q, int OPS>
static hipError_t launch_t(const pa_op *op, int variant, const double *x, double *y, const int32_t *elist, int n,
                           hipStream_t s)
{
    switch (variant) {
    case PA_VARIANT_VALU: return launch_k<D, Q, OPS, EX_VALU64, true>(op, op->d_qdata, x, y, elist, n, s);
    case PA_VARIANT_MFMA_COLORED: return launch_k<D, Q, OPS, EX_MFMA64, false>(op, op->d_qdata, x, y, elist, n, s);
    default: return launch_k<D, Q, OPS, EX_MFMA64, true>(op, op->d_qdata, x, y, elist, n, s);
    }
}

template <int D, int Q, int OPS>
static hipError_t launch_t_lp(const pa_op *op, int fmt, const float *x, float *y, hipStream_t s)
{
    if (fmt == PA_LP_BF16) return launch_k<D, Q, OPS, EX_MFMA16B, true>(op, op->d_qdata32, x, y, nullptr, op->nelem, s);
    return launch_k<D, Q, OPS, EX_MFMA16F, true>(op, op->d_qdata32, x, y, nullptr, op->nelem, s);
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

template <int P>
static hipError_t launch_p_lp(const pa_op *op, int fmt, const float *x, float *y, hipStream_t s, bool *ok)
{
    constexpr int D = P + 1;
    *ok = true;
    if (op->q == P + 1) {
        switch (op->ops) {
        case 1: return launch_t_lp<D, P + 1, 1>(op, fmt, x, y, s);
        case 2: return launch_t_lp<D, P + 1, 2>(op, fmt, x, y, s);
        case 3: return launch_t_lp<D, P + 1, 3>(op, fmt, x, y, s);
        }
    } else if (op->q == P + 2) {
        switch (op->ops) {
        case 1: return launch_t_lp<D, P + 2, 1>(op, fmt, x, y, s);
        case 2: return launch_t_lp<D, P + 2, 2>(op, fmt, x, y, s);
        case 3: return launch_t_lp<D, P + 2, 3>(op, fmt, x, y, s);
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
hipError_t HEXPA_CAT(launch_apply_lp_p, HEXPA_APPLY_P)(const pa_op *op, int fmt, const float *x, float *y,
                                                      hipStream_t s, bool *ok)
{
    return launch_p_lp<HEXPA_APPLY_P>(op, fmt, x, y, s, ok);
}

}  // namespace hexpa
