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
#include "geometry.h"

namespace hexpa {

// Workgroup barrier for LDS traffic only.  __syncthreads() also orders global memory at
// workgroup scope, which on gfx950 means s_waitcnt vmcnt(0) before every barrier: every
// prefetched map/x load and every scatter atomic in flight would be waited for.  The
// waves of a workgroup exchange data only through LDS, so waiting for LDS (lgkmcnt) is
// enough; loads whose registers are used later are still waited for by the compiler.
__device__ __forceinline__ void lds_barrier() { asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory"); }

constexpr int kMinWavesPerEU = 3;  // register budget: waves resident per SIMD

// Contraction executors.
enum : int { EX_MFMA64 = 0, EX_VALU64 = 1, EX_MFMA16F = 2, EX_MFMA16B = 3 };
template <int EX>
struct ExT {
    using T = typename std::conditional<(EX >= EX_MFMA16F), float, double>::type;
};

template <class S>
struct GroupRegs {
    static constexpr int NM = (S::E * S::D3 + S::THREADS - 1) / S::THREADS;  // map/x slots per thread
};

// LDS position of local node I = i + D (j + D k) in the padded input X[n=(j,k)][i]
template <class S>
__device__ __forceinline__ int xpos(int I)
{
    return I + (S::DP - S::ND) * (I / S::ND);
}
// Centre every staged x tile on its element mean (the BF16 diffusion apply).  Diffusion
// annihilates constants element by element (the reference gradients of the basis sum to
// zero), so y_E is unchanged in exact arithmetic, while the 16-bit rounding of the tile at
// the MFMA input now acts on the deviation from the mean instead of the full values: for a
// smooth x this removes the error term proportional to u |mean| (at the 32^3, p = 6 mixed
// workload: 16x smaller error for a smooth x in BF16, 10x in FP16).  One wave per element
// forms the mean (FP32, fixed order); two LDS barriers, ~7 % of the apply.  FP16 keeps the
// plain tile: its reliable-update solve was no faster with centring.
template <class S, int E, int NT, class T>
__device__ __forceinline__ void centre_tiles(T *bufA, T *emean, int tid)
{
    const int wave = tid >> 6, lane = tid & 63;
    for (int e = wave; e < E; e += NT / 64) {
        T sum = T(0);
        for (int I = lane; I < S::D3; I += 64) sum += bufA[e * S::SZ_A + xpos<S>(I)];
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off);
        if (lane == 0) emean[e] = sum / T(S::D3);
    }
    lds_barrier();
    for (int L = tid; L < E * S::D3; L += NT) {
        const int e = L / S::D3, I = L - e * S::D3;
        bufA[e * S::SZ_A + xpos<S>(I)] -= emean[e];
    }
    lds_barrier();
}

// LDS position of entry r of the natural quadrature-point tensor [channel][Q^3]
template <int Q, bool M>
__device__ __forceinline__ int qtpos(int r)
{
    const int ch = r / (Q * Q * Q);
    return ch * Chan<Q, M>::CS + Chan<Q, M>::qpos(r - ch * Q * Q * Q);
}

// Workgroup size, LDS budget and register budget (waves per SIMD) of the register-staged
// kernel, measured per order.  Diffusion at p <= 4 runs two-wave workgroups (fewer waves
// wait at each barrier, more workgroups per CU): a 24 KB element budget at p = 4 (two
// elements), 16 KB at p <= 2 with at least six waves per SIMD (p = 2: 2.59 -> 2.49 ms at
// 155^3; the smaller groups put seven workgroups on a CU instead of five).  The mass
// operator at p <= 2 with Q = p + 2 keeps four waves but a 20 KB budget and six waves per
// SIMD (p = 2: 0.94 -> 0.74 ms: a group's arithmetic is small against its D, map and x
// traffic, so what hides the memory latency is the number of groups in flight per CU, six,
// not three; at p = 3, at Q = p + 1 and in the matrix-free stage that register budget
// would spill).  Everything else: four waves, 48 KB, three waves per SIMD.
template <int D, int Q, int OPS, int EX, int STAGE = 0>
struct ApplyCfg {
    static constexpr bool SMALL = (OPS & 2) != 0 && D <= 5 && (EX == 0 || EX == 1);
    static constexpr bool DIFF_LO = SMALL && D <= 3 && STAGE == 0;
    static constexpr bool MASS_LO = OPS == 1 && D <= 3 && Q == D + 1 && (EX == 0 || EX == 1) && STAGE == 0;
    static constexpr int NT = SMALL ? 128 : kThreads;
    static constexpr int BUDGET = DIFF_LO ? 16 * 1024 : SMALL ? 24 * 1024 : MASS_LO ? 20 * 1024 : kLdsBudget;
    static constexpr int MINW = DIFF_LO || MASS_LO ? 6 : kMinWavesPerEU;
};

// D of one group into registers: slot s of thread tid is qp entry L = tid + s*THREADS.
// EL: the launch passes an element list (only the coloured launches do).  Making it a
// compile-time property keeps the list loads, and the memory waits their results need,
// out of every other instance.
template <class S, bool EL, class T>
__device__ __forceinline__ void load_qdata(T (&dq)[S::NS][S::NCOMP], const T *__restrict__ qd,
                                           const int32_t *__restrict__ elist, int e0, int nv, int tid)
{
#pragma unroll
    for (int s = 0; s < S::NS; ++s) {
        const int L = tid + s * S::THREADS;
        const int e = L / S::Q3, r = L - e * S::Q3;
        const bool ok = e < nv;
        const int64_t ge = ok ? (EL ? elist[e0 + e] : e0 + e) : 0;
        const T *src = qd + ge * (int64_t)(S::NCOMP * S::Q3) + r;
#pragma unroll
        for (int c = 0; c < S::NCOMP; ++c) dq[s][c] = ok ? __builtin_nontemporal_load(src + c * S::Q3) : T(0);
    }
}

template <class S, bool EL>
__device__ __forceinline__ void load_map(int32_t (&m)[GroupRegs<S>::NM], const int32_t *__restrict__ emap,
                                         const int32_t *__restrict__ elist, int e0, int nv, int tid)
{
#pragma unroll
    for (int s = 0; s < GroupRegs<S>::NM; ++s) {
        const int L = tid + s * S::THREADS;
        int e, I;
        row_node<S::ND, S::E>(L, e, I);
        int32_t gi = -1;
        if (L < S::E * S::D3 && e < nv) {
            const int64_t ge = EL ? elist[e0 + e] : e0 + e;
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

// One contraction pass with the chosen executor.  MFMA A-operands come from the basis
// blocks held in registers (ab, when Q is a multiple of 4) or are read from the LDS copy of
// the tables right before the pass; the VALU executor reads the tables with uniform loads
// from global memory.
template <class P, int E, int EX, int NT, class T, class Out, class AB>
__device__ __forceinline__ void run_pass(const T *in, int szin, const DevTables *stab, const DevTables *gtab,
                                         const Out &out, int tid, const AB &ab)
{
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    if constexpr (EX == EX_MFMA64) {
        double a[PassRegs<P>::RT][PassRegs<P>::KC];
        if constexpr (AB::on && AB::template direct<P>())
            ab.template view<P>(a);
        else
            load_a<P>(stab, a, lane);
        mfma_pass<P, E, NT>(in, szin, a, out, wave, lane);
    } else if constexpr (EX == EX_VALU64) {
        valu_pass<P, E, NT>(in, szin, gtab, out, tid);
    } else {
        constexpr bool BF = EX == EX_MFMA16B;
        typename Mfma16<BF>::V a[PassRegs16<P>::RB][PassRegs16<P>::KC];
        if constexpr (AB::on && AB::template direct<P>())
            ab.template view<P>(a);
        else
            load_a16<P, BF>(stab, a, lane);
        mfma16_pass<P, E, NT, BF>(in, szin, a, out, wave, lane);
    }
}

// Basis blocks in registers (ABlocks): both for the whole kernel where they fit, else each
// for its half of every group.  The two passes whose matrix does not start on a whole tile
// of a block when Q is not a multiple of 4 (dz forward, dx transposed) then run as wide
// passes on the whole block, so no pass keeps tiles of its own beside the block (with per-
// pass tiles beside it the p = 8 diffusion kernel needed 144 registers and lost a wave per
// SIMD: 1.32 -> 1.48 ms).  WideIf picks the pass to run: its wide form when it would take
// its tiles from a block it does not start on.
template <class AB, class P, class PW>
using WideIf = typename std::conditional<AB::wide_ok && !AB::template direct<P>(), PW, P>::type;
// the block type of an executor: FP64 tiles, 16-bit tiles (always small), or none (VALU)
template <int D, int Q, int OPS, int EX, bool ON>
using ABlocksFor = typename std::conditional<
    EX == EX_MFMA64, ABlocks<D, Q, ON>,
    typename std::conditional<(EX >= EX_MFMA16F), ABlocks16<D, Q, EX == EX_MFMA16B, ON>,
                              ABlocks<D, Q, false>>::type>::type;

// STAGE 0: the fused apply.  The unfused apply (the paper's baseline that fusion is
// measured against) runs the same code in three launches through HBM: STAGE 1 gathers x,
// runs the forward contractions and writes the quadrature-point tensor of every element to
// qbuf [e][channel][Q^3]; k_dstep applies D there in place; STAGE 2 reads it back, runs the
// transposed contractions and scatters into y.  STAGE 3 is the fused matrix-free apply:
// no stored D; the D-step recomputes it at every quadrature point from the element's eight
// vertices (staged in LDS per group) and the coefficient, with the setup kernel's code.
template <int D, int Q, int OPS, int EX, bool ATOMIC, int STAGE = 0>
__global__ __launch_bounds__((ApplyCfg<D, Q, OPS, EX, STAGE>::NT), (ApplyCfg<D, Q, OPS, EX, STAGE>::MINW)) void k_apply(
    int nelem, int ngroups, const int32_t *__restrict__ elist, const int32_t *__restrict__ emap,
    const typename ExT<EX>::T *__restrict__ qd, const DevTables *__restrict__ tab,
    const typename ExT<EX>::T *__restrict__ x, typename ExT<EX>::T *__restrict__ y,
    typename ExT<EX>::T *__restrict__ qbuf, const double *__restrict__ vert, const int32_t *__restrict__ hex,
    CoeffDev cf)
{
    using T = typename ExT<EX>::T;
    using CFG = ApplyCfg<D, Q, OPS, EX, STAGE>;
    using S = Shape<D, Q, OPS, (int)sizeof(T), CFG::NT, CFG::BUDGET>;
    constexpr int NT = S::THREADS;
    constexpr int E = S::E, D3 = S::D3, Q3 = S::Q3, NS = S::NS, NC = S::NCOMP, NM = GroupRegs<S>::NM;
    constexpr bool M = S::kMass;
    constexpr bool EL = !ATOMIC;  // only the coloured (plain read-modify-write) launches pass an element list
    // two-wave workgroups: the independent y-direction passes (forward: on B x and on G x;
    // transposed: the two paths) each get a wave of their own instead of sharing wave 0
    constexpr bool PAIRS = NT == 128 && S::kDiff;
    __shared__ T bufA[E * S::SZ_A + S::SLACK];
    __shared__ T bufB[E * S::SZ_B + S::SLACK];
    __shared__ int32_t lmap[E * D3];
    __shared__ DevTables stab;  // 1-D tables in LDS: MFMA A-operands are re-read per pass
    constexpr bool CENTRE = EX == EX_MFMA16B && OPS == 2;
    __shared__ T emean[CENTRE ? E : 1];

    const int tid = threadIdx.x;
    for (int i = tid; i < (int)(sizeof(DevTables) / sizeof(double)); i += NT)
        reinterpret_cast<double *>(&stab)[i] = reinterpret_cast<const double *>(tab)[i];
    // (not in the matrix-free stage, whose geometry work already fills the registers)
    ABlocksFor<D, Q, OPS, EX, STAGE != 3> ab;
    ab.kernel_start(tab, tid & 63);

    // Workgroup b runs on XCD b % 8.  XCD x owns the contiguous group range
    // [G x / 8, G (x+1) / 8) so neighbouring elements (sharing DOFs of x and y) meet in the
    // same L2; its workgroups take that range's groups round-robin.  The two-wave diffusion
    // instances instead stride over all groups in launch order (neighbouring groups on
    // different XCDs), measured 4-5 % faster for them at p = 2..4; the four-wave instances
    // keep the XCD ranges (p = 4 mass 2.5 % faster with them).
    // (Grids of fewer than 8 workgroups just stride over all groups.)
    const int nb = gridDim.x;
    int g, gend, nbx;
    if (!CFG::SMALL && nb >= 8) {
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

    constexpr bool FWD = STAGE != 2, MF = STAGE == 3, DSTEP = STAGE == 0 || MF, LOADD = STAGE == 0;
    __shared__ double vxs[MF ? E * 24 : 1];  // vertex coordinates of the group's elements (MF)
    constexpr int QT = S::NG * Q3;  // quadrature-point tensor per element (unfused stages)
    T dq[NS][NC];
    int32_t mcur[NM];
    T xcur[NM];
    {
        const int e0 = g * E, nv = min(E, nelem - e0);
        if constexpr (LOADD) load_qdata<S, EL>(dq, qd, elist, e0, nv, tid);
        load_map<S, EL>(mcur, emap, elist, e0, nv, tid);
        if constexpr (FWD) load_x<S>(xcur, mcur, x);
    }

    for (;;) {
        const int e0 = g * E, nv = min(E, nelem - e0);
        const int gn = g + nbx;
        const bool more = gn < gend;
        const int e0n = gn * E, nvn = more ? min(E, nelem - e0n) : 0;

        // stage x_E = G_e x (local node order = X[e][n=(j,k)][i]) and the map
#pragma unroll
        for (int s = 0; s < NM; ++s) {
            const int L = tid + s * NT;
            if (L < E * D3) {
                int e, I;
                row_node<D, E>(L, e, I);
                lmap[e * D3 + I] = mcur[s];
                if constexpr (FWD) bufA[e * S::SZ_A + xpos<S>(I)] = xcur[s];
            }
        }
        if constexpr (MF)
            for (int L = tid; L < nv * 24; L += NT) {
                const int e = L / 24, c = (L - e * 24) / 3, r = L - e * 24 - 3 * c;
                const int64_t ge = EL ? elist[e0 + e] : e0 + e;
                vxs[L] = vert[(int64_t)hex[ge * 8 + c] * 3 + r];
            }
        if constexpr (!FWD)  // the quadrature-point tensor, D already applied by k_dstep
            for (int L = tid; L < nv * QT; L += NT) {
                const int e = L / QT, r = L - e * QT;
                bufB[e * S::SZ_B + qtpos<Q, M>(r)] = qbuf[(int64_t)(e0 + e) * QT + r];
            }
        int32_t mnext[NM];
        load_map<S, EL>(mnext, emap, elist, e0n, nvn, tid);
        lds_barrier();
        if constexpr (CENTRE && FWD) centre_tiles<S, E, NT>(bufA, emean, tid);

        // forward contractions
        ab.forward_start(&stab, tid & 63);
        if constexpr (!FWD) {
        } else if constexpr (S::kDiff) {
            run_pass<DF1<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            lds_barrier();
            if constexpr (PAIRS) {  // the two independent y passes on one wave each
                if (tid < 64)
                    run_pass<DF2a<D, Q, M>, E, EX, 64>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
                else
                    run_pass<DF2b<D, Q, M>, E, EX, 64>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid - 64, ab);
            } else {
                run_pass<DF2a<D, Q, M>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
                run_pass<DF2b<D, Q, M>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            }
            lds_barrier();
            run_pass<WideIf<decltype(ab), DF3a<D, Q, M>, DF3aW<D, Q, M>>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            run_pass<DF3b<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            run_pass<DF3c<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
        } else {
            run_pass<MF1<D, Q>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            lds_barrier();
            run_pass<MF2<D, Q>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            lds_barrier();
            run_pass<MF3<D, Q>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
        }
        // the next group's map has had the forward passes to arrive: start its x gather
        T xnext[NM];
        if constexpr (FWD) load_x<S>(xnext, mnext, x);
        lds_barrier();
        if constexpr (STAGE == 1) {  // the quadrature-point tensor goes to HBM; next group
            for (int L = tid; L < nv * QT; L += NT) {
                const int e = L / QT, r = L - e * QT;
                qbuf[(int64_t)(e0 + e) * QT + r] = bufB[e * S::SZ_B + qtpos<Q, M>(r)];
            }
            if (!more) break;
            lds_barrier();
            g = gn;
#pragma unroll
            for (int s = 0; s < NM; ++s) {
                mcur[s] = mnext[s];
                xcur[s] = xnext[s];
            }
            continue;
        }

        // D at quadrature points: v = D grad_ref u (symmetric 3x3) and/or v_u = D_m u
#pragma unroll
        for (int s = 0; s < (DSTEP ? NS : 0); ++s) {
            const int L = tid + s * NT;
            if (L < E * Q3) {
                const int e = L / Q3, r = L - e * Q3;
                T *V = bufB + e * S::SZ_B + Chan<Q, M>::qpos(r);
                T dmf[MF ? NC : 1];
                if constexpr (MF) {
                    Hex h;
#pragma unroll
                    for (int c = 0; c < 8; ++c)
#pragma unroll
                        for (int k = 0; k < 3; ++k) h.X[c][k] = vxs[e * 24 + 3 * c + k];
                    const int qa = r % Q, qb = (r / Q) % Q, qc = r / (Q * Q);
                    qp_data<OPS>(h, stab.x[qa], stab.x[qb], stab.x[qc], stab.w[qa] * stab.w[qb] * stab.w[qc], cf, dmf);
                }
                const T *Dm = MF ? dmf : dq[s];
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
        if (LOADD && more) load_qdata<S, EL>(dq, qd, elist, e0n, nvn, tid);  // the next group's D
        lds_barrier();

        // transposed contractions and scatter-add
        ab.transposed_start(&stab, tid & 63);
        if constexpr (S::kDiff) {
            using CH = Chan<Q, M>;
            run_pass<WideIf<decltype(ab), DT1<D, Q, M, CH::X, 0, true>, DT1W<D, Q, M, CH::X, 0>>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            run_pass<DT1<D, Q, M, CH::Y, 1, false>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            run_pass<DT1<D, Q, M, CH::Z, 2, false>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            if constexpr (M)
                run_pass<DT1<D, Q, M, CH::V, 3, false>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A},
                                                                tid, ab);
            lds_barrier();
            if constexpr (PAIRS) {
                if (tid < 64)
                    run_pass<DT2a<D, Q, M>, E, EX, 64>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
                else
                    run_pass<DT2b<D, Q, M>, E, EX, 64>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid - 64, ab);
            } else {
                run_pass<DT2a<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
                run_pass<DT2b<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            }
            lds_barrier();
            run_pass<DT3<D, Q, M>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
        } else {
            run_pass<MT1<D, Q>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            lds_barrier();
            run_pass<MT2<D, Q>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            lds_barrier();
            run_pass<MT3<D, Q>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
        }
        lds_barrier();
        scatter_group<D, E, NT, S::SZ_A, ATOMIC>(bufA, lmap, y, tid);
        if (!more) break;
        lds_barrier();  // LDS (X, map) is rewritten by the next group
        g = gn;
#pragma unroll
        for (int s = 0; s < NM; ++s) {
            mcur[s] = mnext[s];
            if constexpr (FWD) xcur[s] = xnext[s];
        }
    }
}

// D-step of the unfused apply, in place on the quadrature-point tensor [e][channel][Q^3]
// (channels as in the fused kernel: dx, dy, (u,) dz for diffusion; u for mass).
template <int Q, int OPS, class T>
__global__ __launch_bounds__(256) void k_dstep(int64_t npts, const T *__restrict__ qd, T *__restrict__ qbuf)
{
    using S = Shape<2, Q, OPS, (int)sizeof(T)>;  // channel counts only (independent of D)
    constexpr int Q3 = Q * Q * Q, NG = S::NG, NC = S::NCOMP;
    constexpr bool M = S::kMass;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npts; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = i / Q3;
        const int r = (int)(i - e * Q3);
        T *V = qbuf + e * (NG * Q3) + r;
        const T *Dm = qd + e * (NC * Q3) + r;
        if constexpr (S::kDiff) {
            using CH = Chan<Q, M>;  // channel c of the natural tensor at c Q^3
            constexpr int X = CH::NX * Q3, Y = CH::NY * Q3, Z = CH::NZ * Q3, U = CH::NV * Q3;
            const T g0 = V[X], g1 = V[Y], g2 = V[Z];
            const T d0 = Dm[0], d1 = Dm[Q3], d2 = Dm[2 * Q3], d3 = Dm[3 * Q3], d4 = Dm[4 * Q3], d5 = Dm[5 * Q3];
            V[X] = d0 * g0 + d1 * g1 + d2 * g2;
            V[Y] = d1 * g0 + d3 * g1 + d4 * g2;
            V[Z] = d2 * g0 + d4 * g1 + d5 * g2;
            if constexpr (M) V[U] = Dm[6 * Q3] * V[U];
        } else {
            V[0] *= Dm[0];
        }
    }
}

// ------------------------------------------------------------------ DMA-staged variant
// Every global load of the element loop goes straight into LDS (global_load_lds: 16 bytes
// per lane for D, 4 bytes per lane for the DOF map and for the two halves of each
// gathered x value), issued from inline assembly so that the compiler neither waits for
// them nor counts them; the kernel waits for all of them at one point per group, the
// D-step, where D is needed anyway.  Per group g:
//   stage x(g) from LDS | issue x(g+1) (map(g+1) already in LDS) and map(g+2) |
//   forward passes | wait, D-step | issue D(g+1) | transposed passes and scatter.
// So the D stream of the next group overlaps the transposed passes and the forward
// passes, and the gathers overlap the forward passes, without holding registers.
constexpr int kDmaMinD = 6;                // orders p >= 5 (measured faster there; diffusion at p <= 4 keeps the register kernel)
constexpr int kDmaLdsBudget = 53 * 1024;   // LDS bytes per workgroup of the DMA kernel

__device__ __forceinline__ uint32_t lds_byte_addr(const void *p)
{
    return (uint32_t)(uintptr_t)(const __attribute__((address_space(3))) void *)p;
}
// lane l writes [base + size l, base + size (l + 1)) of LDS; base is made wave-uniform.
// M0 (the LDS base register of these loads) is saved and restored inside the statement.
__device__ __forceinline__ void dma4(const void *src, uint32_t base)
{
    uint32_t saved;
    asm volatile(
        "s_mov_b32 %0, m0\n\ts_mov_b32 m0, %2\n\ts_nop 0\n\tglobal_load_lds_dword %1, off\n\ts_mov_b32 m0, %0"
        : "=&s"(saved)
        : "v"(src), "s"(__builtin_amdgcn_readfirstlane(base))
        : "memory");
}
__device__ __forceinline__ void dma_wait() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// D goes to registers (loaded after the D-step for the next group); the DOF map and the
// gathered x go to LDS.
template <int D, int Q, int OPS, class T>
struct DmaShape {
    using B = Shape<D, Q, OPS, (int)sizeof(T)>;
    static constexpr int TB = (int)sizeof(T);
    static constexpr int PER = TB * (B::SZ_A + B::SZ_B) + 12 * B::D3 + (TB == 8 ? 8 : 4) * B::D3;
    // buffer tails for the padding columns of 16-column tiles (the exact bound: a smaller
    // footprint leaves room for more workgroups per CU)
    static constexpr int SLACK = 16 * cmax(B::DP, B::QP);
    static constexpr int FIXED = TB * 2 * SLACK + (int)sizeof(DevTables);
    // the mass operator: a 40 KB budget and four waves per SIMD, so four workgroups share
    // a CU instead of three (p = 4: 0.529 -> 0.485 ms at 78^3, p = 6: 0.481 -> 0.470 ms);
    // the 16-bit diffusion apply at p = 6: one element per group and five waves per SIMD,
    // five workgroups per CU instead of four (Q = 8: 0.194 -> 0.182 ms at 32^3; at p = 5
    // and 7 that register budget would spill)
    static constexpr bool LP = TB == 4 && OPS == 2 && D == 7;
    static constexpr int BUDGET = OPS == 1 ? 40 * 1024 : LP ? 26 * 1024 : kDmaLdsBudget;
    static constexpr int E = cclamp((BUDGET - FIXED) / PER, 1, 32);
    // the mass operator from p = 4 (0.565 -> 0.529 ms at 78^3; at p = 2 the register
    // kernel stays faster: 0.94 against 0.99 ms before either had its occupancy setting,
    // 0.75 ms now)
    static constexpr bool ok = D >= kDmaMinD || (OPS == 1 && D >= 5);
    // one element per group at p = 8: eight waves share it (each pass has 6-7 column tiles)
    static constexpr int NT = (E == 1 && D >= 9) ? 512 : kThreads;
    static constexpr int MINW = NT == 512 ? 2 : OPS == 1 ? 4 : LP ? 5 : kMinWavesPerEU;
};

template <int D, int Q, int OPS, int EX, bool ATOMIC>
__global__ __launch_bounds__((DmaShape<D, Q, OPS, typename ExT<EX>::T>::NT),
                             (DmaShape<D, Q, OPS, typename ExT<EX>::T>::MINW)) void k_apply_dma(
    int nelem, int ngroups, const int32_t *__restrict__ elist, const int32_t *__restrict__ emap,
    const typename ExT<EX>::T *__restrict__ qd, const DevTables *__restrict__ tab,
    const typename ExT<EX>::T *__restrict__ x, typename ExT<EX>::T *__restrict__ y)
{
    using T = typename ExT<EX>::T;
    using S = Shape<D, Q, OPS, (int)sizeof(T)>;
    constexpr int NT = DmaShape<D, Q, OPS, T>::NT;
    constexpr int E = DmaShape<D, Q, OPS, T>::E, D3 = S::D3, Q3 = S::Q3, NC = S::NCOMP, ED3 = E * D3;
    constexpr int NSD = (E * Q3 + NT - 1) / NT;
    constexpr bool M = S::kMass, WIDE = sizeof(T) == 8;
    constexpr bool EL = !ATOMIC;  // only the coloured (plain read-modify-write) launches pass an element list
    T dq[NSD][NC];
    __shared__ T bufA[E * S::SZ_A + DmaShape<D, Q, OPS, T>::SLACK];
    __shared__ T bufB[E * S::SZ_B + DmaShape<D, Q, OPS, T>::SLACK];
    __shared__ int32_t mapb[3][ED3];
    __shared__ uint32_t XL[ED3], XH[WIDE ? ED3 : 1];
    __shared__ DevTables stab;
    constexpr bool CENTRE = EX == EX_MFMA16B && OPS == 2;
    __shared__ T emean[CENTRE ? E : 1];

    const int tid = threadIdx.x, lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int i = tid; i < (int)(sizeof(DevTables) / sizeof(double)); i += NT)
        reinterpret_cast<double *>(&stab)[i] = reinterpret_cast<const double *>(tab)[i];
    ABlocksFor<D, Q, OPS, EX, true> ab;
    ab.kernel_start(tab, tid & 63);

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

    // map of group gg into buffer b (absent element slots get -1)
    auto issue_map = [&](int gg, int b) {
        const int e0 = gg * E, nv = min(E, nelem - e0);
        for (int L0 = wave * 64; L0 < ED3; L0 += NT) {
            const int L = L0 + lane;
            const uint32_t base = lds_byte_addr(&mapb[b][L0]);
            if (L < nv * D3) {
                const int e = L / D3, I = L - e * D3;
                const int64_t ge = EL ? elist[e0 + e] : e0 + e;
                dma4(emap + ge * D3 + I, base);
            } else if (L < ED3) {
                mapb[b][L] = -1;
            }
        }
    };
    // x gathered through the map in buffer b (absent slots read x[0], never scattered)
    auto issue_x = [&](int b) {
        for (int L0 = wave * 64; L0 < ED3; L0 += NT) {
            const int L = L0 + lane;
            const uint32_t bl = lds_byte_addr(&XL[L0]);
            const uint32_t bh = WIDE ? lds_byte_addr(&XH[L0]) : 0u;
            if (L < ED3) {
                const int m = mapb[b][L];
                const T *src = x + (m >= 0 ? m : 0);
                dma4(src, bl);
                if constexpr (WIDE) dma4(reinterpret_cast<const char *>(src) + 4, bh);
            }
        }
    };
    auto issue_d = [&](int gg) {  // into registers: slot s of thread tid is qp entry tid + s NT
        const int e0 = gg * E, nv = min(E, nelem - e0);
#pragma unroll
        for (int s = 0; s < NSD; ++s) {
            const int L = tid + s * NT;
            const int e = L / Q3, r = L - e * Q3;
            const bool ok = e < nv;
            const int64_t ge = ok ? (EL ? elist[e0 + e] : e0 + e) : 0;
            const T *src = qd + ge * (int64_t)(NC * Q3) + r;
#pragma unroll
            for (int c = 0; c < NC; ++c) dq[s][c] = ok ? __builtin_nontemporal_load(src + c * Q3) : T(0);
        }
    };

    // prologue: maps of the first two groups, D of the first, then its x
    issue_map(g, 0);
    if (g + nbx < gend) issue_map(g + nbx, 1);
    issue_d(g);
    dma_wait();
    lds_barrier();
    issue_x(0);
    dma_wait();
    lds_barrier();

    int mb = 0;  // buffer holding this group's map
    for (;;) {
        const int gn = g + nbx, gn2 = gn + nbx;
        const bool more = gn < gend, more2 = gn2 < gend;
        const int mb1 = mb == 2 ? 0 : mb + 1, mb2 = mb1 == 2 ? 0 : mb1 + 1;

        // stage x_E from the gathered halves
        for (int L = tid; L < ED3; L += NT) {
            const int e = L / D3, I = L - e * D3;
            T v;
            if constexpr (WIDE) v = __hiloint2double((int)XH[L], (int)XL[L]);
            else v = __uint_as_float(XL[L]);
            bufA[e * S::SZ_A + xpos<S>(I)] = v;
        }
        lds_barrier();
        if (more) issue_x(mb1);
        if (more2) issue_map(gn2, mb2);
        if constexpr (CENTRE) centre_tiles<S, E, NT>(bufA, emean, tid);

        // forward contractions
        ab.forward_start(&stab, tid & 63);
        if constexpr (S::kDiff) {
            run_pass<DF1<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            lds_barrier();
            run_pass<DF2a<D, Q, M>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            run_pass<DF2b<D, Q, M>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            lds_barrier();
            run_pass<WideIf<decltype(ab), DF3a<D, Q, M>, DF3aW<D, Q, M>>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            run_pass<DF3b<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            run_pass<DF3c<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
        } else {
            run_pass<MF1<D, Q>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            lds_barrier();
            run_pass<MF2<D, Q>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            lds_barrier();
            run_pass<MF3<D, Q>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
        }
        // D of this group, the next group's x and the map after it have landed
        dma_wait();
        lds_barrier();

#pragma unroll
        for (int s = 0; s < NSD; ++s) {
            const int L = tid + s * NT;
            if (L < E * Q3) {
                const int e = L / Q3, r = L - e * Q3;
                T *V = bufB + e * S::SZ_B + Chan<Q, M>::qpos(r);
                T dv[NC];
#pragma unroll
                for (int c = 0; c < NC; ++c) dv[c] = dq[s][c];
                if constexpr (S::kDiff) {
                    using CH = Chan<Q, M>;
                    const T g0 = V[CH::X], g1 = V[CH::Y], g2 = V[CH::Z];
                    V[CH::X] = dv[0] * g0 + dv[1] * g1 + dv[2] * g2;
                    V[CH::Y] = dv[1] * g0 + dv[3] * g1 + dv[4] * g2;
                    V[CH::Z] = dv[2] * g0 + dv[4] * g1 + dv[5] * g2;
                    if constexpr (M) V[CH::V] = dv[6] * V[CH::V];
                } else {
                    V[0] *= dv[0];
                }
            }
        }
        lds_barrier();
        if (more) issue_d(gn);

        // transposed contractions and scatter-add
        ab.transposed_start(&stab, tid & 63);
        const int32_t *lmap = mapb[mb];
        if constexpr (S::kDiff) {
            using CH = Chan<Q, M>;
            run_pass<WideIf<decltype(ab), DT1<D, Q, M, CH::X, 0, true>, DT1W<D, Q, M, CH::X, 0>>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            run_pass<DT1<D, Q, M, CH::Y, 1, false>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            run_pass<DT1<D, Q, M, CH::Z, 2, false>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            if constexpr (M)
                run_pass<DT1<D, Q, M, CH::V, 3, false>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A},
                                                                tid, ab);
            lds_barrier();
            run_pass<DT2a<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            run_pass<DT2b<D, Q, M>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            lds_barrier();
            run_pass<DT3<D, Q, M>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
        } else {
            run_pass<MT1<D, Q>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
            lds_barrier();
            run_pass<MT2<D, Q>, E, EX, NT>(bufA, S::SZ_A, &stab, tab, LdsOut<T>{bufB, S::SZ_B}, tid, ab);
            lds_barrier();
            run_pass<MT3<D, Q>, E, EX, NT>(bufB, S::SZ_B, &stab, tab, LdsOut<T>{bufA, S::SZ_A}, tid, ab);
        }
        lds_barrier();
        scatter_group<D, E, NT, S::SZ_A, ATOMIC>(bufA, lmap, y, tid);
        if (!more) break;
        lds_barrier();  // bufA, XL/XH and the oldest map buffer are rewritten next
        g = gn;
        mb = mb1;
    }
    // no load is left in flight at exit: the last group issued none after its wait
}

// ------------------------------------------------------------------ launchers
// grid of a persistent kernel: resident capacity (queried once per kernel: the template
// parameter is the kernel itself, so each has its own cached value), at most ngroups
template <auto KERN>
static int persistent_blocks(int nt, int ngroups)
{
    const auto kern = KERN;
    static int cap = 0;
    if (cap == 0) {
        int per_cu = 0, dev = 0, ncu = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, nt, 0) != hipSuccess || per_cu < 1) per_cu = 1;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1)
            ncu = 256;
        cap = per_cu * ncu;
    }
    return ngroups < cap ? ngroups : cap;
}

// grid of an apply launch: the persistent grid, capped by pa_set_grid_cap
static int capped(const pa_op *op, int nblocks)
{
    return (op->grid_cap > 0 && op->grid_cap < nblocks) ? op->grid_cap : nblocks;
}

// The unfused apply: forward stage, D-step, transposed stage (y must hold zeros).
template <int D, int Q, int OPS, int EX>
static hipError_t launch_unfused(const pa_op *op, const double *x, double *y, double *qbuf, hipStream_t s)
{
    using CFG = ApplyCfg<D, Q, OPS, EX, 1>;
    using S = Shape<D, Q, OPS, 8, CFG::NT, CFG::BUDGET>;
    const int n = op->nelem;
    const int ngroups = (n + S::E - 1) / S::E;
    if (ngroups == 0) return hipSuccess;
    constexpr auto k1 = k_apply<D, Q, OPS, EX, true, 1>;
    constexpr auto k3 = k_apply<D, Q, OPS, EX, true, 2>;
    hipLaunchKernelGGL(k1, dim3(capped(op, persistent_blocks<k1>(CFG::NT, ngroups))), dim3(CFG::NT), 0, s, n, ngroups,
                       (const int32_t *)nullptr, op->d_elem_dofs, op->d_qdata, op->d_tab, x, y, qbuf, op->d_vert,
                       op->d_hex, op->coeff);
    const int64_t npts = (int64_t)n * S::Q3;
    auto k2 = k_dstep<Q, OPS, double>;
    hipLaunchKernelGGL(k2, dim3((unsigned)std::min<int64_t>((npts + 255) / 256, 65536)), dim3(256), 0, s, npts,
                       (const double *)op->d_qdata, qbuf);
    hipLaunchKernelGGL(k3, dim3(capped(op, persistent_blocks<k3>(CFG::NT, ngroups))), dim3(CFG::NT), 0, s, n, ngroups,
                       (const int32_t *)nullptr, op->d_elem_dofs, op->d_qdata, op->d_tab, x, y, qbuf, op->d_vert,
                       op->d_hex, op->coeff);
    return hipGetLastError();
}

// The fused matrix-free apply (D recomputed in the kernel; y must hold zeros).
template <int D, int Q, int OPS, int EX>
static hipError_t launch_mf(const pa_op *op, const double *x, double *y, hipStream_t s)
{
    using CFG = ApplyCfg<D, Q, OPS, EX, 3>;
    using S = Shape<D, Q, OPS, 8, CFG::NT, CFG::BUDGET>;
    const int n = op->nelem;
    const int ngroups = (n + S::E - 1) / S::E;
    if (ngroups == 0) return hipSuccess;
    constexpr auto k = k_apply<D, Q, OPS, EX, true, 3>;
    hipLaunchKernelGGL(k, dim3(capped(op, persistent_blocks<k>(CFG::NT, ngroups))), dim3(CFG::NT), 0, s, n, ngroups,
                       (const int32_t *)nullptr, op->d_elem_dofs, op->d_qdata, op->d_tab, x, y, (double *)nullptr,
                       op->d_vert, op->d_hex, op->coeff);
    return hipGetLastError();
}

template <int D, int Q, int OPS, int EX, bool ATOMIC>
static hipError_t launch_k(const pa_op *op, const typename ExT<EX>::T *qd, const typename ExT<EX>::T *x,
                           typename ExT<EX>::T *y, const int32_t *elist, int n, hipStream_t s)
{
    using T = typename ExT<EX>::T;
    using CFG = ApplyCfg<D, Q, OPS, EX>;
    constexpr bool DMA = DmaShape<D, Q, OPS, T>::ok;
    // elements per group and workgroup size exactly as the chosen kernel computes them
    constexpr int EG = DMA ? DmaShape<D, Q, OPS, T>::E : Shape<D, Q, OPS, (int)sizeof(T), CFG::NT, CFG::BUDGET>::E;
    constexpr int NT = DMA ? DmaShape<D, Q, OPS, T>::NT : CFG::NT;
    const int ngroups = (n + EG - 1) / EG;
    if (ngroups == 0) return hipSuccess;
    if constexpr (!DMA) {
        constexpr auto kern = k_apply<D, Q, OPS, EX, ATOMIC, 0>;
        const int nblocks = capped(op, persistent_blocks<kern>(NT, ngroups));
        hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), 0, s, n, ngroups, elist, op->d_elem_dofs, qd, op->d_tab, x,
                           y, (T *)nullptr, (const double *)nullptr, (const int32_t *)nullptr, CoeffDev{});
    } else {
        constexpr auto kern = k_apply_dma<D, Q, OPS, EX, ATOMIC>;
        const int nblocks = capped(op, persistent_blocks<kern>(NT, ngroups));
        hipLaunchKernelGGL(kern, dim3(nblocks), dim3(NT), 0, s, n, ngroups, elist, op->d_elem_dofs, qd, op->d_tab, x,
                           y);
    }
    return hipGetLastError();
}

template <int D, int Q, int OPS>
static hipError_t launch_t(const pa_op *op, int variant, const double *x, double *y, const int32_t *elist, int n,
                           double *qbuf, hipStream_t s)
{
    switch (variant) {
    case PA_VARIANT_MFMA_UNFUSED: return launch_unfused<D, Q, OPS, EX_MFMA64>(op, x, y, qbuf, s);
    case PA_VARIANT_VALU_UNFUSED: return launch_unfused<D, Q, OPS, EX_VALU64>(op, x, y, qbuf, s);
    case PA_VARIANT_MFMA_MF: return launch_mf<D, Q, OPS, EX_MFMA64>(op, x, y, s);
    case PA_VARIANT_VALU_MF: return launch_mf<D, Q, OPS, EX_VALU64>(op, x, y, s);
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
                           double *qbuf, hipStream_t s, bool *ok)
{
    constexpr int D = P + 1;
    *ok = true;
    if (op->q == P + 1) {
        switch (op->ops) {
        case 1: return launch_t<D, P + 1, 1>(op, variant, x, y, elist, n, qbuf, s);
        case 2: return launch_t<D, P + 1, 2>(op, variant, x, y, elist, n, qbuf, s);
        case 3: return launch_t<D, P + 1, 3>(op, variant, x, y, elist, n, qbuf, s);
        }
    } else if (op->q == P + 2) {
        switch (op->ops) {
        case 1: return launch_t<D, P + 2, 1>(op, variant, x, y, elist, n, qbuf, s);
        case 2: return launch_t<D, P + 2, 2>(op, variant, x, y, elist, n, qbuf, s);
        case 3: return launch_t<D, P + 2, 3>(op, variant, x, y, elist, n, qbuf, s);
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

// elements per group and workgroup size of the kernel a launch of this variant runs
template <int D, int Q, int OPS, int EX, bool FUSED_STORED>
static void group_shape(int *elems, int *threads)
{
    using T = typename ExT<EX>::T;
    using CFG = ApplyCfg<D, Q, OPS, EX, FUSED_STORED ? 0 : 1>;
    constexpr bool DMA = FUSED_STORED && DmaShape<D, Q, OPS, T>::ok;
    *elems = DMA ? DmaShape<D, Q, OPS, T>::E : Shape<D, Q, OPS, (int)sizeof(T), CFG::NT, CFG::BUDGET>::E;
    *threads = DMA ? DmaShape<D, Q, OPS, T>::NT : CFG::NT;
}

template <int D, int Q, int OPS>
static void group_shape_t(int variant, int *elems, int *threads)
{
    switch (variant) {
    case PA_VARIANT_MFMA_UNFUSED:
    case PA_VARIANT_MFMA_MF: return group_shape<D, Q, OPS, EX_MFMA64, false>(elems, threads);
    case PA_VARIANT_VALU_UNFUSED:
    case PA_VARIANT_VALU_MF: return group_shape<D, Q, OPS, EX_VALU64, false>(elems, threads);
    case PA_VARIANT_VALU: return group_shape<D, Q, OPS, EX_VALU64, true>(elems, threads);
    case -1: return group_shape<D, Q, OPS, EX_MFMA16F, true>(elems, threads);  // the 16-bit apply
    default: return group_shape<D, Q, OPS, EX_MFMA64, true>(elems, threads);
    }
}

template <int P>
static bool group_shape_p(int q, int ops, int variant, int *elems, int *threads)
{
    constexpr int D = P + 1;
    if (q != P + 1 && q != P + 2) return false;
    if (ops < 1 || ops > 3) return false;
    if (q == P + 1) {
        if (ops == 1) group_shape_t<D, P + 1, 1>(variant, elems, threads);
        if (ops == 2) group_shape_t<D, P + 1, 2>(variant, elems, threads);
        if (ops == 3) group_shape_t<D, P + 1, 3>(variant, elems, threads);
    } else {
        if (ops == 1) group_shape_t<D, P + 2, 1>(variant, elems, threads);
        if (ops == 2) group_shape_t<D, P + 2, 2>(variant, elems, threads);
        if (ops == 3) group_shape_t<D, P + 2, 3>(variant, elems, threads);
    }
    return true;
}

#ifndef HEXPA_APPLY_P
#error "compile k_apply.hip once per order with -DHEXPA_APPLY_P=<p>"
#endif

#define HEXPA_CAT2(a, b) a##b
#define HEXPA_CAT(a, b) HEXPA_CAT2(a, b)
hipError_t HEXPA_CAT(launch_apply_p, HEXPA_APPLY_P)(const pa_op *op, int variant, const double *x, double *y,
                                                   const int32_t *elist, int n, double *qbuf, hipStream_t s, bool *ok)
{
    return launch_p<HEXPA_APPLY_P>(op, variant, x, y, elist, n, qbuf, s, ok);
}
hipError_t HEXPA_CAT(launch_apply_lp_p, HEXPA_APPLY_P)(const pa_op *op, int fmt, const float *x, float *y,
                                                      hipStream_t s, bool *ok)
{
    return launch_p_lp<HEXPA_APPLY_P>(op, fmt, x, y, s, ok);
}
bool HEXPA_CAT(apply_group_shape_p, HEXPA_APPLY_P)(int q, int ops, int variant, int *elems, int *threads)
{
    return group_shape_p<HEXPA_APPLY_P>(q, ops, variant, elems, threads);
}

}  // namespace hexpa
