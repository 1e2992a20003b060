// Fused PA apply for H1 mass / diffusion on hexahedra: shared device machinery.
//
// One workgroup (256 threads = 4 wave64) owns a group of E elements and runs, for all of
// them at once:
//   gather x_E = G_e x  ->  forward contractions (B, and its derivative G for diffusion)
//   -> D at quadrature points -> transposed contractions -> scatter-add y += G_e^T y_E.
// This is the operator A = G^T B^T D B G of the paper's eq. (1) with the tensor contraction
// of eq. (2) split into three one-index contractions (Sec. III-D).
//
// Every contraction stage ("pass") is, per element, a small GEMM
//     Out[o][n] = sum_k A[o][k] * In[n][k]
// where k runs over the contracted 1-D index (and, for K-stacked passes, over several
// input tensors that feed the same output), n over the two untouched indices, and o over
// the new 1-D index.  The paper's cyclic index order (Sec. III-D) is what makes this
// uniform: storing each stage's output as [o][n] leaves the next stage's contracted index
// fastest in memory, so the input of every pass is In[n][k] with unit stride in k (and an
// odd column stride, see the LDS layout below).
//
// Two executors consume the same pass descriptors:
//   * MFMA: v_mfma_f64_4x4x4f64 (four 4x4x4 blocks = a 4x16x4 GEMM slice) with A (the
//     1-D basis) as the A-operand in VGPRs, 16 GEMM columns (n, across the E elements)
//     per tile as the B-operand read from LDS, and 4 output rows per row tile;
//   * VALU: one thread per GEMM column, all O outputs in registers, A read with uniform
//     (scalar) loads.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "internal.h"

namespace hexpa {

constexpr int kThreads = 256;  // threads per workgroup of the fused apply (four-wave instances)
constexpr int kWaves = kThreads / 64;
constexpr int kLdsBudget = 48 * 1024;  // bytes of LDS per workgroup for the element tensors
constexpr int kMfmaBatch = 2;          // MFMA tiles in flight per wave
constexpr int kValuBatch = 2;          // GEMM columns in flight per thread

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmax3(int a, int b, int c) { return cmax(a, cmax(b, c)); }
constexpr int cclamp(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }
// LDS column stride of a tensor whose fast index has length c: 8-byte reads of 16 lanes
// (one LDS cycle) at a stride of c doubles fall on gcd(c, 16) times fewer banks than a
// conflict-free read needs, so strides that are multiples of 4 (4- and 8-way conflicts)
// are padded by one; the 2-way conflict of c = 2 mod 4 costs less than the footprint.
__host__ __device__ constexpr int pad_stride(int c) { return c % 4 == 0 ? c + 1 : c; }

// ------------------------------------------------------------------ element-group shape
// TB: bytes of the LDS/vector scalar type; NT: threads per workgroup; BUDGET: LDS bytes per
// workgroup for the element tensors
template <int D, int Q, int OPS, int TB = 8, int NT = kThreads, int BUDGET = kLdsBudget>
struct Shape {
    static constexpr int THREADS = NT;
    static constexpr bool kMass = (OPS & 1) != 0;
    static constexpr bool kDiff = (OPS & 2) != 0;
    static constexpr int NCOMP = kDiff ? (kMass ? 7 : 6) : 1;  // stored D values per qp
    static constexpr int NG = kDiff ? (kMass ? 4 : 3) : 1;     // qp channels (grad comps, value)
    static constexpr int ND = D, NQ = Q;  // 1-D node and quadrature-point counts
    static constexpr int Q3 = Q * Q * Q, D3 = D * D * D;
    // element tensors with the fast index stored at stride DP = pad_stride(D) or QP = pad_stride(Q)
    static constexpr int DP = pad_stride(D), QP = pad_stride(Q);
    static constexpr int SZ_X = D * D * DP;
    static constexpr int SZ_U1 = (kDiff ? 2 * Q : Q) * D * DP;
    static constexpr int SZ_U2 = (kDiff ? 3 * Q * Q : Q * Q) * DP;
    static constexpr int SZ_G3 = NG * Q * Q * QP;
    static constexpr int SZ_W = NG * Q * QP * D;
    static constexpr int SZ_T = (kDiff ? 2 : 1) * D * D * QP;
    // ping-pong LDS regions per element (doubles); odd strides spread elements over banks
    static constexpr int SZ_A = cmax3(SZ_X, SZ_U2, SZ_W) | 1;
    static constexpr int SZ_B = cmax3(SZ_U1, SZ_G3, SZ_T) | 1;
    // tail of each buffer read by the padding columns of the last element's 16-column tiles
    // (at most 15 columns past the element region at column stride <= max(DP, QP); the
    // larger fixed size keeps the measured workgroups-per-CU of every order)
    static constexpr int SLACK = 16 * 2 * kMaxQ;
    static constexpr int PER_ELEM_BYTES = TB * (SZ_A + SZ_B) + 4 * D3;
    // elements per workgroup from the LDS budget (48 KB -> 3 workgroups per 160 KB CU)
    static constexpr int E = cclamp(BUDGET / PER_ELEM_BYTES, 1, 32);
    static constexpr int NS = (E * Q3 + NT - 1) / NT;  // qp slots per thread
};

// ------------------------------------------------------------------ scatter
// Scatter-add of a group's element outputs y_E (staged in LDS, natural node order per
// element at stride SZ) through the DOF map.  Consecutive elements of a group are usually
// neighbours along x (elements are ordered x fastest): the right face (i = D-1) of element
// e and the left face (i = 0) of element e+1 then hold the same DOFs, and their two
// contributions are summed here so that each such DOF gets one global addition instead of
// two.  Whether the faces coincide is read from the map itself (equal DOF numbers), so
// any element order and mesh stay exact; only the merging opportunity depends on it.
// Lanes walk the group in row order (node row (j,k), then element, then i), so a wave's
// atomics cover runs of consecutive DOFs across the group's elements instead of D-long
// pieces of many rows: FP64 atomics are executed beyond the L2 per cache line requested,
// and this order cuts the lines per instruction several-fold (measured: the mass apply
// 1.2-1.45x faster at p = 2..6).
template <int D, int E, int NT, int SZ, bool ATOMIC, class T>
__device__ __forceinline__ void scatter_group(const T *stage, const int32_t *lmap, T *y, int tid)
{
    constexpr int D3 = D * D * D, ROW = E * D;
    for (int R = tid; R < E * D3; R += NT) {
        const int jk = R / ROW, t = R - jk * ROW;
        const int e = t / D, i = t - e * D;
        const int I = i + D * jk, L = e * D3 + I;
        const int32_t g = lmap[L];
        if (g < 0) continue;
        if (i == 0 && e > 0 && lmap[L - D3 + (D - 1)] == g) continue;  // added by the left neighbour
        T v = stage[e * SZ + I];
        if (i == D - 1 && e + 1 < E && lmap[L + D3 - (D - 1)] == g) v += stage[(e + 1) * SZ + I - (D - 1)];
        if (ATOMIC)
            unsafeAtomicAdd(y + g, v);
        else
            y[g] += v;
    }
}

// Row order of a group's nodes (row (j,k), then element, then i): slot R -> element e and
// local node I = i + D (j + D k).  The register kernel gathers x in this order, so the
// lanes of one load read consecutive DOFs of a row across the group's elements.
template <int D, int E>
__device__ __forceinline__ void row_node(int R, int &e, int &I)
{
    constexpr int ROW = E * D;
    const int jk = R / ROW, t = R - jk * ROW;
    e = t / D;
    I = t - e * D + D * jk;
}

// ------------------------------------------------------------------ table accessors
__device__ __forceinline__ double tB(const DevTables *t, int a, int i, int D) { return t->B[a * D + i]; }
__device__ __forceinline__ double tG(const DevTables *t, int a, int i, int D) { return t->G[a * D + i]; }

// ------------------------------------------------------------------ MFMA executor
// v_mfma_f64_4x4x4f64 computes four independent 4x4x4 products; block beta = (l>>2)&3
// takes its A-operand from lane l as A_beta[l&3][l>>4], its B-operand as B_beta[l>>4][l&3]
// and returns D_beta[l>>4][l&3] in lane l (pinned by test_mfma_f64_lane_layouts).  With
// the same A in every block, the four blocks are one 4 (rows) x 16 (columns) x 4 (k) GEMM
// slice: column n = l & 15, contracted index k = l >> 4, output row l >> 4.  On gfx950
// this shape sustains ~1.4x the FP64 rate of v_mfma_f64_16x16x4f64 and pads the small
// 1-D dimensions (d = p+1, Q) to multiples of 4 instead of 16.
// Optional members of a "wide" pass (one that takes a whole basis block although it needs
// only part of it): KREG register k length, ROFF the first register row it stores and OS how
// many, KOFF the register k of its first input column and KS how many input columns.
template <class P, class = void>
struct PassX {
    static constexpr int KREG = P::NT * P::C, ROFF = 0, OS = P::O, KOFF = 0, KS = P::NT * P::C;
};
template <class P>
struct PassX<P, std::void_t<decltype(P::KREG)>> {
    static constexpr int KREG = P::KREG, ROFF = P::ROFF, OS = P::OS, KOFF = P::KOFF, KS = P::KS;
};

template <class P>
struct PassRegs {
    static constexpr int K = PassX<P>::KREG;
    static constexpr int KC = (K + 3) / 4;   // k chunks of 4
    static constexpr int RT = (P::O + 3) / 4;  // 4-row tiles
};

// A operand: lane l holds A[4 rt + (l & 3)][4 kc + (l >> 4)] of the stacked pass matrix.
template <class P>
__device__ __forceinline__ void load_a(const DevTables *tab, double (&a)[PassRegs<P>::RT][PassRegs<P>::KC], int lane)
{
    constexpr int K = PassRegs<P>::K;
#pragma unroll
    for (int rt = 0; rt < PassRegs<P>::RT; ++rt)
#pragma unroll
        for (int kc = 0; kc < PassRegs<P>::KC; ++kc) {
            const int o = 4 * rt + (lane & 3);
            const int k = 4 * kc + (lane >> 4);
            a[rt][kc] = (o < P::O && k < K) ? P::A(tab, o, k) : 0.0;
        }
}

// The 1-D basis as MFMA A-operands in registers (FP64 MFMA executor).  Most pass matrices
// are whole 4x4 tiles of one of two blocks
//   F = [B; G]      rows o < Q: B[o][k], Q <= o < 2Q: G[o-Q][k]; k < D (forward passes),
//   T = [B^T G^T]   rows o < D; k < Q: B[k][o], Q <= k < 2Q: G[k-Q][o] (transposed passes)
// (pass row tile rt is block tile amrt(rt), k chunk kc is amkc(kc)).  When Q is not a
// multiple of 4 the G-only passes do not start on a tile; the kernels then run them as
// wide passes on the whole block (DF3aW, DT1W), and only the mass term's third K-stacked
// tensor (AV false) still reads its tiles from the LDS tables per pass.  Where both blocks
// fit (p <= 6) they stay in registers for the whole kernel; at larger p F is read from the
// LDS tables at the start of each group's forward passes and T at the start of its
// transposed ones.  Either way the tables are read once per group and wave instead of once
// per pass: at p = 6 that removes about 40 % of the kernel's LDS instructions (counters).
// Lane l holds A[4 rt + (l & 3)][4 kc + (l >> 4)] as in load_a, so the results are those
// of the per-pass loads.
template <int D, int Q, bool ON>
struct ABlocks {
    static constexpr bool on = ON, wide_ok = ON;
    static constexpr int RTF = ON ? (2 * Q + 3) / 4 : 1, KCF = ON ? (D + 3) / 4 : 1;
    static constexpr int RTT = ON ? (D + 3) / 4 : 1, KCT = ON ? (2 * Q + 3) / 4 : 1;
    // both blocks for the whole kernel, or each for its half of every group
    static constexpr bool WHOLE = RTF * KCF + RTT * KCT <= 16;
    double f[RTF][KCF], t[RTT][KCT];
    __device__ __forceinline__ void load_f(const DevTables *tab, int lane)
    {
        if constexpr (ON) {
            const int r = lane & 3, c = lane >> 4;
#pragma unroll
            for (int rt = 0; rt < RTF; ++rt)
#pragma unroll
                for (int kc = 0; kc < KCF; ++kc) {
                    const int o = 4 * rt + r, k = 4 * kc + c;
                    const bool ok = k < D && o < 2 * Q;
                    const int ob = ok ? (o < Q ? o : o - Q) : 0, kk = ok ? k : 0;
                    const double v = o < Q ? tB(tab, ob, kk, D) : tG(tab, ob, kk, D);
                    f[rt][kc] = ok ? v : 0.0;
                }
        }
    }
    __device__ __forceinline__ void load_t(const DevTables *tab, int lane)
    {
        if constexpr (ON) {
            const int r = lane & 3, c = lane >> 4;
#pragma unroll
            for (int rt = 0; rt < RTT; ++rt)
#pragma unroll
                for (int kc = 0; kc < KCT; ++kc) {
                    const int o = 4 * rt + r, k = 4 * kc + c;
                    const bool ok = o < D && k < 2 * Q;
                    const int kb = ok ? (k < Q ? k : k - Q) : 0, oo = ok ? o : 0;
                    const double v = k < Q ? tB(tab, kb, oo, D) : tG(tab, kb, oo, D);
                    t[rt][kc] = ok ? v : 0.0;
                }
        }
    }
    // once per kernel (WHOLE) or at the start of each group's forward / transposed passes
    __device__ __forceinline__ void kernel_start(const DevTables *tab, int lane)
    {
        if constexpr (ON && WHOLE) {
            load_f(tab, lane);
            load_t(tab, lane);
        }
    }
    __device__ __forceinline__ void forward_start(const DevTables *tab, int lane)
    {
        if constexpr (ON && !WHOLE) load_f(tab, lane);
    }
    __device__ __forceinline__ void transposed_start(const DevTables *tab, int lane)
    {
        if constexpr (ON && !WHOLE) load_t(tab, lane);
    }
    // pass P takes its tiles from a block
    template <class P>
    static constexpr bool direct()
    {
        return P::AV;
    }
    // the A-operand tiles of pass P
    template <class P>
    __device__ __forceinline__ void view(double (&a)[PassRegs<P>::RT][PassRegs<P>::KC]) const
    {
#pragma unroll
        for (int rt = 0; rt < PassRegs<P>::RT; ++rt)
#pragma unroll
            for (int kc = 0; kc < PassRegs<P>::KC; ++kc)
                if constexpr (P::AM == 0)
                    a[rt][kc] = f[P::amrt(rt)][P::amkc(kc)];
                else
                    a[rt][kc] = t[P::amrt(rt)][P::amkc(kc)];
    }
};

// Store policy of a pass output (LDS; the last pass stages y_E there for scatter_group).
// `addr` is element-local (OUT + opos(n) + NCOLO o; the last pass writes the natural
// node order n + D^2 o).
template <class T>
struct LdsOut {
    T *out;
    int sz;
    __device__ __forceinline__ void put(int e, int addr, T v) const { out[e * sz + addr] = v; }
};

// LDS layout.  Every per-element tensor is stored with its fast (next-contracted) index
// at the padded stride DP = pad_stride(D) or QP = pad_stride(Q), so that threads or MFMA
// lanes reading consecutive columns (column stride CS) spread over the LDS banks.  A pass
// reads In[n][c] at in_off(t) + n CS + c (c < C) and writes Out[o][n] at
// OUT + opos(n) + NCOLO o, where opos places the fast part f of n = f + OF s at f + OSTR s:
// the layout the next pass reads with column stride OSTR.  The last pass writes the
// element's natural node order (OF = OSTR = NCOL) through the DOF map.
template <class P>
struct OutLayout {
    static constexpr int NCOLO = P::OSTR * (P::NCOL / P::OF);
    __device__ static int opos(int n) { return P::OF == P::OSTR ? n : (n % P::OF) + P::OSTR * (n / P::OF); }
};

// Columns are padded to NCOLP (a multiple of 16) per element so that a 16-column tile
// never straddles two elements: tile t covers element t / TPE, columns
// n0 = 16 (t % TPE) .. n0 + 15.  Tiles are dealt to the waves round-robin; the tile
// index is wave-uniform, so the element/column bases are scalar values and each lane
// adds one lane-constant offset per tile -- no per-element index arithmetic.  Padding
// columns (n >= NCOL) read inside the buffer slack and are never stored.
template <class P>
struct Tiling {
    static constexpr int NCOLP = (P::NCOL + 15) / 16 * 16;
    static constexpr int TPE = NCOLP / 16;
};

template <class P, int E, int NT, class Out>
__device__ __forceinline__ void mfma_pass(const double *in, int szin,
                                          const double (&a)[PassRegs<P>::RT][PassRegs<P>::KC],
                                          const Out &out, int wave, int lane)
{
    constexpr int C = P::C, CS = P::CS, K = PassRegs<P>::K, KC = PassRegs<P>::KC, RT = PassRegs<P>::RT;
    constexpr int TPE = Tiling<P>::TPE, NTILE = E * TPE, NW = NT / 64, NCOLO = OutLayout<P>::NCOLO;
    constexpr int NR = (NTILE + NW - 1) / NW;
    constexpr int BATCH = NR < kMfmaBatch ? NR : kMfmaBatch;
    const int kl = lane >> 4, nl = lane & 15;
    // lane constants: B-operand offsets per k chunk, output offset of row kl
    constexpr int KOFF = PassX<P>::KOFF, KS = PassX<P>::KS, ROFF = PassX<P>::ROFF, OS = PassX<P>::OS;
    int lin[KC];
    bool kval[KC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        const int k = 4 * kc + kl - KOFF;  // input column of register k
        kval[kc] = k >= 0 && k < KS;
        const int kk = kval[kc] ? k : 0;
        const int t = kk / C, c = kk - t * C;
        lin[kc] = nl * CS + (kval[kc] ? P::in_off(t) + c : 0);
    }
    const int lout = P::OUT + NCOLO * (kl - ROFF);
#pragma unroll 1
    for (int r0 = 0; r0 < NR; r0 += BATCH) {
        double bv[BATCH][KC];
        int eS[BATCH], n0S[BATCH];
        bool cv[BATCH];
#pragma unroll
        for (int bi = 0; bi < BATCH; ++bi) {
            const int t = wave + NW * (r0 + bi);  // wave-uniform
            const bool tv = (r0 + bi < NR) && t < NTILE;
            const int e = tv ? t / TPE : 0;
            const int n0 = tv ? (t - e * TPE) * 16 : 0;
            eS[bi] = e;
            n0S[bi] = n0;
            cv[bi] = tv && (n0 + nl < P::NCOL);
            // past K a lane reads a value of its own column and zeroes it (a pass that takes
            // its A tiles from a basis block may see nonzero A there); padding columns are
            // independent and never stored
            const double *base = in + e * szin + n0 * CS;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                const double v = base[lin[kc]];
                bv[bi][kc] = kval[kc] ? v : 0.0;
            }
        }
        double acc[BATCH][RT];
#pragma unroll
        for (int bi = 0; bi < BATCH; ++bi)
#pragma unroll
            for (int rt = 0; rt < RT; ++rt) acc[bi][rt] = 0.0;
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int bi = 0; bi < BATCH; ++bi)
#pragma unroll
                for (int rt = 0; rt < RT; ++rt)
                    acc[bi][rt] = __builtin_amdgcn_mfma_f64_4x4x4f64(a[rt][kc], bv[bi][kc], acc[bi][rt], 0, 0, 0);
#pragma unroll
        for (int bi = 0; bi < BATCH; ++bi) {
            if (!cv[bi]) continue;
            const int ob = lout + OutLayout<P>::opos(n0S[bi] + nl);
#pragma unroll
            for (int rt = 0; rt < RT; ++rt)
                if (4 * rt + kl >= ROFF && 4 * rt + kl < ROFF + OS) out.put(eS[bi], ob + 4 * rt * NCOLO, acc[bi][rt]);
        }
    }
}

// ------------------------------------------------------------------ VALU executor
// One thread per GEMM column, all O outputs in registers.  BATCH columns per thread are
// loaded before any FMA so the LDS latency of one hides behind another.
template <class P, int E, int NTH, class Out>
__device__ __forceinline__ void valu_pass(const double *in, int szin, const DevTables *tab, const Out &out, int tid)
{
    static_assert(PassX<P>::KOFF == 0 && PassX<P>::ROFF == 0, "wide passes are FP64 MFMA only");
    constexpr int C = P::C, CS = P::CS, NT = P::NT, O = P::O, NCOLO = OutLayout<P>::NCOLO;
    constexpr int NCOLS = E * P::NCOL;
    constexpr int NR = (NCOLS + NTH - 1) / NTH;
    constexpr int BATCH = NR < kValuBatch ? NR : kValuBatch;
#pragma unroll 1
    for (int r0 = 0; r0 < NR; r0 += BATCH) {
        double xin[BATCH][NT * C];
        int eI[BATCH], nI[BATCH];
        bool cv[BATCH];
#pragma unroll
        for (int bi = 0; bi < BATCH; ++bi) {
            int col = tid + NTH * (r0 + bi);
            cv[bi] = (r0 + bi < NR) && col < NCOLS;
            if (!cv[bi]) col = 0;
            eI[bi] = col / P::NCOL;
            nI[bi] = col - eI[bi] * P::NCOL;
            const double *base = in + eI[bi] * szin + nI[bi] * CS;
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int c = 0; c < C; ++c) xin[bi][t * C + c] = base[P::in_off(t) + c];
        }
#pragma unroll
        for (int bi = 0; bi < BATCH; ++bi) {
            double acc[O];
#pragma unroll
            for (int o = 0; o < O; ++o) acc[o] = 0.0;
#pragma unroll
            for (int k = 0; k < NT * C; ++k)
#pragma unroll
                for (int o = 0; o < O; ++o) acc[o] = fma(P::A(tab, o, k), xin[bi][k], acc[o]);
            if (cv[bi]) {
                const int ob = P::OUT + OutLayout<P>::opos(nI[bi]);
#pragma unroll
                for (int o = 0; o < O; ++o) out.put(eI[bi], ob + NCOLO * o, acc[o]);
            }
        }
    }
}

// ------------------------------------------------------------------ 16-bit MFMA executor
// v_mfma_f32_16x16x16{f16,bf16}: lane l supplies A[l%16][4(l/16)+t] and B[4(l/16)+t][l%16]
// (t = 0..3, four 16-bit values) and returns D[4(l/16)+v][l%16] (v = 0..3, FP32),
// pinned by test_mfma_16bit_lane_layouts.  Used by the mixed-precision inner apply: the
// LDS tensors hold FP32 values that are rounded to FP16/BF16 as they enter the MFMA,
// and the products accumulate in FP32.
// The B-operand needs no masking: a lane whose k lies past the pass's K reads a real
// (finite) value of its own column, and the A-operand is zero there; a padding column
// (past NCOL, or an idle tile) may read stale LDS, but GEMM columns are independent and
// those outputs are never stored.
typedef _Float16 half4_t __attribute__((ext_vector_type(4)));
typedef short bf16x4_t __attribute__((ext_vector_type(4)));
typedef float flt4_t __attribute__((ext_vector_type(4)));
typedef float flt2_t __attribute__((ext_vector_type(2)));
typedef _Float16 half2_t __attribute__((ext_vector_type(2)));
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
typedef unsigned u32x2_t __attribute__((ext_vector_type(2)));

template <bool BF>
struct Mfma16 {
    using V = typename std::conditional<BF, bf16x4_t, half4_t>::type;
    // four FP32 values rounded to nearest-even 16-bit, two per v_cvt_pk_{bf16,f16}_f32
    __device__ static __forceinline__ V pack(const float (&f)[4])
    {
        using H2 = typename std::conditional<BF, bf16x2_t, half2_t>::type;
        const H2 lo = __builtin_convertvector((flt2_t{f[0], f[1]}), H2);
        const H2 hi = __builtin_convertvector((flt2_t{f[2], f[3]}), H2);
        const u32x2_t w = {__builtin_bit_cast(unsigned, lo), __builtin_bit_cast(unsigned, hi)};
        return __builtin_bit_cast(V, w);
    }
    __device__ static __forceinline__ flt4_t mma(V a, V b, flt4_t c)
    {
        if constexpr (BF)
            return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
        else
            return __builtin_amdgcn_mfma_f32_16x16x16f16(a, b, c, 0, 0, 0);
    }
};

template <class P>
struct PassRegs16 {
    static constexpr int K = PassX<P>::KREG;
    static constexpr int KC = (K + 15) / 16;   // k chunks of 16
    static constexpr int RB = (P::O + 15) / 16;  // 16-row blocks
};

template <class P, bool BF>
__device__ __forceinline__ void load_a16(const DevTables *tab,
                                         typename Mfma16<BF>::V (&a)[PassRegs16<P>::RB][PassRegs16<P>::KC], int lane)
{
    constexpr int K = PassRegs16<P>::K;
#pragma unroll
    for (int rb = 0; rb < PassRegs16<P>::RB; ++rb)
#pragma unroll
        for (int kc = 0; kc < PassRegs16<P>::KC; ++kc) {
            float f[4];
            const int o = 16 * rb + (lane & 15);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int k = 16 * kc + 4 * (lane >> 4) + t;
                f[t] = (o < P::O && k < K) ? (float)P::A(tab, o, k) : 0.0f;
            }
            a[rb][kc] = Mfma16<BF>::pack(f);
        }
}

// The same basis blocks F = [B; G] and T = [B^T G^T] as 16x16 A-operand tiles of the
// 16-bit MFMA, packed once per kernel (a few registers per block).  A pass uses them when
// its matrix is the leading rows and columns of a block (B-only row blocks run into unstored
// G rows, B^T-only k blocks into zeroed B-operand columns); the others (G-only, and the
// third tensor of the mass term's K-stacked pass) pack their tiles per pass as before.
template <int D, int Q, bool BF, bool ON>
struct ABlocks16 {
    using V = typename Mfma16<BF>::V;
    static constexpr bool on = ON, wide_ok = ON;
    static constexpr int RBF = ON ? (2 * Q + 15) / 16 : 1, KCF = ON ? (D + 15) / 16 : 1;
    static constexpr int RBT = ON ? (D + 15) / 16 : 1, KCT = ON ? (2 * Q + 15) / 16 : 1;
    V f[RBF][KCF], t[RBT][KCT];
    __device__ __forceinline__ void load(const DevTables *tab, int lane)
    {
        if constexpr (ON) {
#pragma unroll
            for (int rb = 0; rb < RBF; ++rb)
#pragma unroll
                for (int kc = 0; kc < KCF; ++kc) {
                    float v4[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int o = 16 * rb + (lane & 15), k = 16 * kc + 4 * (lane >> 4) + u;
                        const bool ok = k < D && o < 2 * Q;
                        const int ob = ok ? (o < Q ? o : o - Q) : 0, kk = ok ? k : 0;
                        const double v = o < Q ? tB(tab, ob, kk, D) : tG(tab, ob, kk, D);
                        v4[u] = ok ? (float)v : 0.0f;
                    }
                    f[rb][kc] = Mfma16<BF>::pack(v4);
                }
#pragma unroll
            for (int rb = 0; rb < RBT; ++rb)
#pragma unroll
                for (int kc = 0; kc < KCT; ++kc) {
                    float v4[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int o = 16 * rb + (lane & 15), k = 16 * kc + 4 * (lane >> 4) + u;
                        const bool ok = o < D && k < 2 * Q;
                        const int kb = ok ? (k < Q ? k : k - Q) : 0, oo = ok ? o : 0;
                        const double v = k < Q ? tB(tab, kb, oo, D) : tG(tab, kb, oo, D);
                        v4[u] = ok ? (float)v : 0.0f;
                    }
                    t[rb][kc] = Mfma16<BF>::pack(v4);
                }
        }
    }
    __device__ __forceinline__ void kernel_start(const DevTables *tab, int lane) { load(tab, lane); }
    __device__ __forceinline__ void forward_start(const DevTables *, int) {}
    __device__ __forceinline__ void transposed_start(const DevTables *, int) {}
    // pass P's matrix is the leading rows and columns of its block
    template <class P>
    static constexpr bool leading()
    {
        if (!P::AV) return false;
        for (int i = 0; i < 16; ++i)
            if (P::amrt(i) != i || P::amkc(i) != i) return false;
        return true;
    }
    template <class P>
    static constexpr bool direct()
    {
        return leading<P>();
    }
    template <class P>
    __device__ __forceinline__ void view(V (&a)[PassRegs16<P>::RB][PassRegs16<P>::KC]) const
    {
#pragma unroll
        for (int rb = 0; rb < PassRegs16<P>::RB; ++rb)
#pragma unroll
            for (int kc = 0; kc < PassRegs16<P>::KC; ++kc)
                if constexpr (P::AM == 0)
                    a[rb][kc] = f[rb][kc];
                else
                    a[rb][kc] = t[rb][kc];
    }
};

template <class P, int E, int NT, bool BF, class Out>
__device__ __forceinline__ void mfma16_pass(const float *in, int szin,
                                            const typename Mfma16<BF>::V (&a)[PassRegs16<P>::RB][PassRegs16<P>::KC],
                                            const Out &out, int wave, int lane)
{
    using V = typename Mfma16<BF>::V;
    constexpr int C = P::C, CS = P::CS, KC = PassRegs16<P>::KC, RB = PassRegs16<P>::RB;
    constexpr int KOFF = PassX<P>::KOFF, KS = PassX<P>::KS, ROFF = PassX<P>::ROFF, OS = PassX<P>::OS;
    constexpr int TPE = Tiling<P>::TPE, NTILE = E * TPE, NW = NT / 64, NCOLO = OutLayout<P>::NCOLO;
    constexpr int NR = (NTILE + NW - 1) / NW;
    constexpr int BATCH = NR < kMfmaBatch ? NR : kMfmaBatch;
    const int kl = lane >> 4, nl = lane & 15;
    int lin[KC][4];
    bool kval[KC][4];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc)
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int k = 16 * kc + 4 * kl + t - KOFF;  // input column of register k
            kval[kc][t] = k >= 0 && k < KS;
            const int kk = kval[kc][t] ? k : 0;
            const int tt = kk / C, c = kk - tt * C;
            lin[kc][t] = nl * CS + (kval[kc][t] ? P::in_off(tt) + c : 0);
        }
    const int lout = P::OUT + NCOLO * (4 * kl - ROFF);
#pragma unroll 1
    for (int r0 = 0; r0 < NR; r0 += BATCH) {
        V bv[BATCH][KC];
        int eS[BATCH], n0S[BATCH];
        bool cv[BATCH];
#pragma unroll
        for (int bi = 0; bi < BATCH; ++bi) {
            const int t = wave + NW * (r0 + bi);
            const bool tv = (r0 + bi < NR) && t < NTILE;
            const int e = tv ? t / TPE : 0;
            const int n0 = tv ? (t - e * TPE) * 16 : 0;
            eS[bi] = e;
            n0S[bi] = n0;
            cv[bi] = tv && (n0 + nl < P::NCOL);
            const float *base = in + e * szin + n0 * CS;
#pragma unroll
            for (int kc = 0; kc < KC; ++kc) {
                float f[4];
#pragma unroll
                for (int t4 = 0; t4 < 4; ++t4) {
                    const float v = base[lin[kc][t4]];
                    f[t4] = kval[kc][t4] ? v : 0.0f;
                }
                bv[bi][kc] = Mfma16<BF>::pack(f);
            }
        }
        flt4_t acc[BATCH][RB];
#pragma unroll
        for (int bi = 0; bi < BATCH; ++bi)
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[bi][rb] = flt4_t{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc)
#pragma unroll
            for (int bi = 0; bi < BATCH; ++bi)
#pragma unroll
                for (int rb = 0; rb < RB; ++rb) acc[bi][rb] = Mfma16<BF>::mma(a[rb][kc], bv[bi][kc], acc[bi][rb]);
#pragma unroll
        for (int bi = 0; bi < BATCH; ++bi) {
            if (!cv[bi]) continue;
            const int ob = lout + OutLayout<P>::opos(n0S[bi] + nl);
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v)
                    if (16 * rb + 4 * kl + v >= ROFF && 16 * rb + 4 * kl + v < ROFF + OS)
                        out.put(eS[bi], ob + NCOLO * (16 * rb + v), acc[bi][rb][v]);
        }
    }
}

}  // namespace hexpa
