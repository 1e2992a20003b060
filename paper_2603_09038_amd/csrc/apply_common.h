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
// fastest in memory, so the input of every pass is In[n][k] with unit stride in k.
//
// Two executors consume the same pass descriptors:
//   * MFMA: v_mfma_f64_16x16x4f64 with A (the 1-D basis) resident in VGPRs as the
//     16x4 A-operand, 16 GEMM columns (n, across the E elements) per tile as the 4x16
//     B-operand read from LDS, and 16 output rows per row block;
//   * VALU: one thread per GEMM column, all O outputs in registers, A read with uniform
//     (scalar) loads.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "internal.h"

namespace hexpa {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;

typedef double dbl4 __attribute__((ext_vector_type(4)));

constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int cmax3(int a, int b, int c) { return cmax(a, cmax(b, c)); }
constexpr int cclamp(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

// ------------------------------------------------------------------ element-group shape
template <int D, int Q, int OPS>
struct Shape {
    static constexpr bool kMass = (OPS & 1) != 0;
    static constexpr bool kDiff = (OPS & 2) != 0;
    static constexpr int NCOMP = kDiff ? (kMass ? 7 : 6) : 1;  // stored D values per qp
    static constexpr int NG = kDiff ? (kMass ? 4 : 3) : 1;     // qp channels (grad comps, value)
    static constexpr int Q3 = Q * Q * Q, D3 = D * D * D;
    static constexpr int SZ_X = D3;
    static constexpr int SZ_U1 = (kDiff ? 2 * Q : Q) * D * D;
    static constexpr int SZ_U2 = (kDiff ? 3 * Q * Q : Q * Q) * D;
    static constexpr int SZ_G3 = NG * Q3;
    static constexpr int SZ_W = NG * Q * Q * D;
    static constexpr int SZ_T = (kDiff ? 2 : 1) * D * D * Q;
    // ping-pong LDS regions per element (doubles); odd strides spread elements over banks
    static constexpr int SZ_A = cmax3(SZ_X, SZ_U2, SZ_W) | 1;
    static constexpr int SZ_B = cmax3(SZ_U1, SZ_G3, SZ_T) | 1;
    static constexpr int PER_ELEM_BYTES = 8 * (SZ_A + SZ_B) + 4 * D3;
    // elements per workgroup: ~48 KB of LDS per group -> 3 groups per CU (160 KB)
    static constexpr int E = cclamp((48 * 1024) / PER_ELEM_BYTES, 1, 32);
    static constexpr int NS = (E * Q3 + kThreads - 1) / kThreads;  // qp slots per thread
};

// ------------------------------------------------------------------ table accessors
__device__ __forceinline__ double tB(const DevTables *t, int a, int i, int D) { return t->B[a * D + i]; }
__device__ __forceinline__ double tG(const DevTables *t, int a, int i, int D) { return t->G[a * D + i]; }

// ------------------------------------------------------------------ MFMA executor
template <class P>
struct PassRegs {
    static constexpr int K = P::NT * P::C;
    static constexpr int KC = (K + 3) / 4;
    static constexpr int RB = (P::O + 15) / 16;
};

// A operand: lane l holds A[rb*16 + l%16][4*kc + l/16] of the stacked pass matrix.
template <class P>
__device__ __forceinline__ void load_a(const DevTables *tab, double (&a)[PassRegs<P>::RB][PassRegs<P>::KC], int lane)
{
    constexpr int K = PassRegs<P>::K;
#pragma unroll
    for (int rb = 0; rb < PassRegs<P>::RB; ++rb)
#pragma unroll
        for (int kc = 0; kc < PassRegs<P>::KC; ++kc) {
            const int o = rb * 16 + (lane & 15);
            const int k = 4 * kc + (lane >> 4);
            a[rb][kc] = (o < P::O && k < K) ? P::A(tab, o, k) : 0.0;
        }
}

// Store policy of a pass output: into LDS, or atomically / plainly into the global y.
struct LdsOut {
    double *out;
    int sz;
    __device__ __forceinline__ void put(int e, int addr, double v) const { out[e * sz + addr] = v; }
};
template <bool ATOMIC>
struct GlobalOut {
    double *y;
    const int32_t *lmap;  // [E][D^3] global index per local node, -1 for absent elements
    int d3;
    __device__ __forceinline__ void put(int e, int addr, double v) const
    {
        const int g = lmap[e * d3 + addr];
        if (g >= 0) {
            if (ATOMIC)
                unsafeAtomicAdd(y + g, v);
            else
                y[g] += v;
        }
    }
};

template <class P, int E, class Out>
__device__ __forceinline__ void mfma_pass(const double *in, int szin,
                                          const double (&a)[PassRegs<P>::RB][PassRegs<P>::KC],
                                          const Out &out, int wave, int lane)
{
    constexpr int C = P::C, K = PassRegs<P>::K, KC = PassRegs<P>::KC, RB = PassRegs<P>::RB;
    constexpr int NTOT = E * P::NCOL;
    constexpr int NTILE = (NTOT + 15) / 16;
    const int kl = lane >> 4, nl = lane & 15;
    int koff[KC];
    bool kval[KC];
#pragma unroll
    for (int kc = 0; kc < KC; ++kc) {
        const int k = 4 * kc + kl;
        kval[kc] = k < K;
        const int t = k / C, c = k - t * C;
        koff[kc] = kval[kc] ? P::in_off(t) + c : 0;
    }
    for (int tile = wave; tile < NTILE; tile += kWaves) {
        const int col = tile * 16 + nl;
        const bool cval = col < NTOT;
        const int e = col / P::NCOL, n = col - e * P::NCOL;
        const double *base = in + e * szin + n * C;
        dbl4 acc[RB];
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) acc[rb] = dbl4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int kc = 0; kc < KC; ++kc) {
            const double b = (cval && kval[kc]) ? base[koff[kc]] : 0.0;
#pragma unroll
            for (int rb = 0; rb < RB; ++rb) acc[rb] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[rb][kc], b, acc[rb], 0, 0, 0);
        }
        if (cval) {
#pragma unroll
            for (int rb = 0; rb < RB; ++rb)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int o = rb * 16 + kl + 4 * v;  // f64 16x16x4 result: row l/16 + 4v
                    if (o < P::O) {
                        const int ad = P::out(o, n);
                        if (ad >= 0) out.put(e, ad, acc[rb][v]);
                    }
                }
        }
    }
}

// ------------------------------------------------------------------ VALU executor
template <class P, int E, class Out>
__device__ __forceinline__ void valu_pass(const double *in, int szin, const DevTables *tab, const Out &out, int tid)
{
    constexpr int C = P::C, NT = P::NT, O = P::O;
    constexpr int NTOT = E * P::NCOL;
    for (int col = tid; col < NTOT; col += kThreads) {
        const int e = col / P::NCOL, n = col - e * P::NCOL;
        const double *base = in + e * szin + n * C;
        double acc[O];
#pragma unroll
        for (int o = 0; o < O; ++o) acc[o] = 0.0;
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const double v = base[P::in_off(t) + c];
#pragma unroll
                for (int o = 0; o < O; ++o) acc[o] = fma(P::A(tab, o, t * C + c), v, acc[o]);
            }
#pragma unroll
        for (int o = 0; o < O; ++o) {
            const int ad = P::out(o, n);
            if (ad >= 0) out.put(e, ad, acc[o]);
        }
    }
}

}  // namespace hexpa
