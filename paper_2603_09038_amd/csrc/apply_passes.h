// Pass descriptors of the fused apply (see apply_common.h for the GEMM convention).
//
// Notation per element: d = D nodes and Q Gauss points per axis; reference-gradient
// channels at a quadrature point (a,b,c) are dx = G_x B_y B_z u, dy = B_x G_y B_z u,
// dz = B_x B_y G_z u and, with the mass term, the value u = B_x B_y B_z u.
//
// Every pass is a plain GEMM per element, Out[o][n] = sum_k A[o][k] In[n][k]:
//   NCOL       GEMM columns per element (the two untouched tensor indices, n),
//   C, NT      length of the contracted index and number of K-stacked input tensors,
//   O          output rows (the new 1-D index; 2Q when the B and G rows are stacked),
//   in_off(t)  offset of input tensor t inside the element's input region (In[n][c] at
//              in_off(t) + n C + c),
//   A(tab,o,k) the stacked pass matrix (k = t C + c),
//   OUT        offset of the output inside the element's output region: Out[o][n] is
//              stored at OUT + n + NCOL o,
//   AV, AM, amrt, amkc  whether the pass's MFMA A-operand tiles are whole 4x4 tiles of one
//              of the two basis blocks that ABlocks keeps in registers, which block, and
//              where (B-only row tiles may run past row Q into the G rows when Q is not a
//              multiple of 4: those rows are computed and never stored; B^T-only k chunks
//              may run into the G^T columns: the pass zeroes its B-operand past K).
// Because each stage stores its output as [o][n], the next stage's contracted index is
// the fastest one in memory (the cyclic index order of the paper's Sec. III-D), and a
// block of rows of one pass (e.g. its G rows) is itself a contiguous tensor.
#pragma once
#include "apply_common.h"

namespace hexpa {

// Channel layout of the quadrature-point tensor V (element region of buffer B), each
// channel [c][b][a] with a at stride QP: dx at 0, dy at QP Q^2; without the mass term dz
// at 2 QP Q^2; with it u at 2 QP Q^2 and dz at 3 QP Q^2.  qpos maps the natural qp index
// r = a + Q (b + Q c) into a channel.
template <int Q, bool M>
struct Chan {
    static constexpr int NX = 0, NY = 1, NV = 2, NZ = M ? 3 : 2;  // channel numbers
    static constexpr int QP = pad_stride(Q), CS = QP * Q * Q;
    static constexpr int X = NX * CS, Y = NY * CS, V = NV * CS, Z = NZ * CS;
    __device__ static int qpos(int r) { return r + (QP - Q) * (r / Q); }
};

// ======================================================================== diffusion
// Forward x: X[n=(j,k)][i] -> U1[o1][n]: rows o1 < Q are B_x X (BX), rows >= Q are G_x X (GX).
template <int D, int Q, bool M>
struct DF1 {
    static constexpr bool AV = true;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D);
    static constexpr int NCOL = D * D, C = D, CS = DP, NT = 1, O = 2 * Q, OUT = 0, OF = D, OSTR = DP;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return o < Q ? tB(t, o, k, D) : tG(t, o - Q, k, D); }
};
// Forward y on BX: BX[n=(k,a)][j] -> rows o2 < Q: T_BB = B_y BX, rows >= Q: T_BG = G_y BX.
template <int D, int Q, bool M>
struct DF2a {
    static constexpr bool AV = true;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D);
    static constexpr int NCOL = Q * D, C = D, CS = DP, NT = 1, O = 2 * Q, OUT = 0, OF = D, OSTR = DP;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return o < Q ? tB(t, o, k, D) : tG(t, o - Q, k, D); }
};
// Forward y on GX: T_GB = B_y GX.
template <int D, int Q, bool M>
struct DF2b {
    static constexpr bool AV = true;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D);
    static constexpr int NCOL = Q * D, C = D, CS = DP, NT = 1, O = Q, OUT = 2 * Q * Q * DP, OF = D, OSTR = DP;
    __device__ static constexpr int in_off(int) { return Q * D * DP; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, D); }
};
// Forward z on T_BB[n=(a,b)][k]: dz = G_z T_BB (and u = B_z T_BB, stacked first, with mass).
template <int D, int Q, bool M>
struct DF3a {
    static constexpr bool AV = M || Q % 4 == 0;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return M ? rt : rt + Q / 4; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D), QP = pad_stride(Q);
    static constexpr int NCOL = Q * Q, C = D, CS = DP, NT = 1, O = M ? 2 * Q : Q, OUT = M ? Chan<Q, M>::V : Chan<Q, M>::Z;
    static constexpr int OF = Q, OSTR = QP;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k)
    {
        return M ? (o < Q ? tB(t, o, k, D) : tG(t, o - Q, k, D)) : tG(t, o, k, D);
    }
};
// Forward z on T_BG: dy = B_z T_BG.
template <int D, int Q, bool M>
struct DF3b {
    static constexpr bool AV = true;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D), QP = pad_stride(Q);
    static constexpr int NCOL = Q * Q, C = D, CS = DP, NT = 1, O = Q, OUT = Chan<Q, M>::Y, OF = Q, OSTR = QP;
    __device__ static constexpr int in_off(int) { return Q * Q * DP; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, D); }
};
// Forward z on T_GB: dx = B_z T_GB.
template <int D, int Q, bool M>
struct DF3c {
    static constexpr bool AV = true;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D), QP = pad_stride(Q);
    static constexpr int NCOL = Q * Q, C = D, CS = DP, NT = 1, O = Q, OUT = Chan<Q, M>::X, OF = Q, OSTR = QP;
    __device__ static constexpr int in_off(int) { return 2 * Q * Q * DP; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, D); }
};
// DF3a without the mass term as a wide pass on the whole [B; G] block (when Q is not a
// multiple of 4 its G rows do not start on a 4-row tile): rows 0..2Q-1 are computed, the G
// rows Q..2Q-1 stored as dz.
template <int D, int Q, bool M>
struct DF3aW {
    static_assert(!M, "with the mass term DF3a already takes the whole block");
    static constexpr bool AV = true;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D), QP = pad_stride(Q);
    static constexpr int NCOL = Q * Q, C = D, CS = DP, NT = 1, O = 2 * Q, OUT = Chan<Q, M>::Z;
    static constexpr int OF = Q, OSTR = QP;
    static constexpr int KREG = D, ROFF = Q, OS = Q, KOFF = 0, KS = D;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return o < Q ? tB(t, o, k, D) : tG(t, o - Q, k, D); }
};
// Transposed x of one channel: V_ch[n=(b,c)][a] -> W_slot[i][n] with G^T (dx) or B^T.
template <int D, int Q, bool M, int CH_OFF, int SLOT, bool GT>
struct DT1 {
    static constexpr bool AV = !GT || Q % 4 == 0;
    static constexpr int AM = 1;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return GT ? kc + Q / 4 : kc; }
    static constexpr int QP = pad_stride(Q);
    static constexpr int NCOL = Q * Q, C = Q, CS = QP, NT = 1, O = D, OUT = SLOT * Q * QP * D, OF = Q, OSTR = QP;
    __device__ static constexpr int in_off(int) { return CH_OFF; }
    __device__ static double A(const DevTables *t, int o, int k) { return GT ? tG(t, k, o, D) : tB(t, k, o, D); }
};
// DT1 with G^T as a wide pass on the whole [B^T G^T] block (when Q is not a multiple of 4 its
// G^T columns do not start on a 4-column chunk): register k Q..2Q-1 carry the channel, the
// B^T columns multiply zeros.
template <int D, int Q, bool M, int CH_OFF, int SLOT>
struct DT1W {
    static constexpr bool AV = true;
    static constexpr int AM = 1;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int QP = pad_stride(Q);
    static constexpr int NCOL = Q * Q, C = Q, CS = QP, NT = 1, O = D, OUT = SLOT * Q * QP * D, OF = Q, OSTR = QP;
    static constexpr int KREG = 2 * Q, ROFF = 0, OS = D, KOFF = Q, KS = Q;
    __device__ static constexpr int in_off(int) { return CH_OFF; }
    __device__ static double A(const DevTables *t, int o, int k) { return k < Q ? tB(t, k, o, D) : tG(t, k - Q, o, D); }
};
// W slots in buffer A: 0 = dx, 1 = dy, 2 = dz, 3 = u.
// Transposed y, path continuing with B_z^T: t1 = B_y^T W0 + G_y^T W1 (+ B_y^T W3).
template <int D, int Q, bool M>
struct DT2a {
    static constexpr bool AV = !M || Q % 4 == 0;
    static constexpr int AM = 1;
    __device__ static constexpr int amrt(int rt) { return rt; }
    // tensors 0, 1 are the B^T, G^T halves of the block; the third (mass, Q a multiple of 4)
    // reuses the B^T half
    __device__ static constexpr int amkc(int kc) { return M ? kc % (Q / 4) + (kc / (Q / 4) == 1 ? Q / 4 : 0) : kc; }
    static constexpr int QP = pad_stride(Q);
    static constexpr int NCOL = Q * D, C = Q, CS = QP, NT = M ? 3 : 2, O = D, OUT = 0, OF = Q, OSTR = QP;
    __device__ static constexpr int in_off(int t) { return (t == 2 ? 3 : t) * Q * QP * D; }
    __device__ static double A(const DevTables *tb, int o, int k)
    {
        const int t = k / Q, b = k - t * Q;
        return t == 1 ? tG(tb, b, o, D) : tB(tb, b, o, D);
    }
};
// Transposed y, path continuing with G_z^T: t2 = B_y^T W2.
template <int D, int Q, bool M>
struct DT2b {
    static constexpr bool AV = true;
    static constexpr int AM = 1;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int QP = pad_stride(Q);
    static constexpr int NCOL = Q * D, C = Q, CS = QP, NT = 1, O = D, OUT = D * D * QP, OF = Q, OSTR = QP;
    __device__ static constexpr int in_off(int) { return 2 * Q * QP * D; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, D); }
};
// Transposed z: y_E[k][n=(i,j)] = B_z^T t1 + G_z^T t2 (K-stacked), scattered to y.
template <int D, int Q, bool M>
struct DT3 {
    static constexpr bool AV = true;
    static constexpr int AM = 1;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int QP = pad_stride(Q);
    static constexpr int NCOL = D * D, C = Q, CS = QP, NT = 2, O = D, OUT = 0, OF = NCOL, OSTR = NCOL;
    __device__ static constexpr int in_off(int t) { return t * D * D * QP; }
    __device__ static double A(const DevTables *tb, int o, int k)
    {
        const int t = k / Q, c = k - t * Q;
        return t == 0 ? tB(tb, c, o, D) : tG(tb, c, o, D);
    }
};

// ======================================================================== mass
template <int D, int Q>
struct MF1 {
    static constexpr bool AV = true;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D);
    static constexpr int NCOL = D * D, C = D, CS = DP, NT = 1, O = Q, OUT = 0, OF = D, OSTR = DP;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, D); }
};
template <int D, int Q>
struct MF2 {
    static constexpr bool AV = true;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D);
    static constexpr int NCOL = Q * D, C = D, CS = DP, NT = 1, O = Q, OUT = 0, OF = D, OSTR = DP;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, D); }
};
template <int D, int Q>
struct MF3 {
    static constexpr bool AV = true;
    static constexpr int AM = 0;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int DP = pad_stride(D), QP = pad_stride(Q);
    static constexpr int NCOL = Q * Q, C = D, CS = DP, NT = 1, O = Q, OUT = 0, OF = Q, OSTR = QP;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, D); }
};
template <int D, int Q>
struct MT1 {
    static constexpr bool AV = true;
    static constexpr int AM = 1;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int QP = pad_stride(Q);
    static constexpr int NCOL = Q * Q, C = Q, CS = QP, NT = 1, O = D, OUT = 0, OF = Q, OSTR = QP;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, D); }
};
template <int D, int Q>
struct MT2 {
    static constexpr bool AV = true;
    static constexpr int AM = 1;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int QP = pad_stride(Q);
    static constexpr int NCOL = Q * D, C = Q, CS = QP, NT = 1, O = D, OUT = 0, OF = Q, OSTR = QP;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, D); }
};
template <int D, int Q>
struct MT3 {
    static constexpr bool AV = true;
    static constexpr int AM = 1;
    __device__ static constexpr int amrt(int rt) { return rt; }
    __device__ static constexpr int amkc(int kc) { return kc; }
    static constexpr int QP = pad_stride(Q);
    static constexpr int NCOL = D * D, C = Q, CS = QP, NT = 1, O = D, OUT = 0, OF = NCOL, OSTR = NCOL;
    __device__ static constexpr int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, D); }
};

}  // namespace hexpa
