// Pass descriptors of the fused apply (see apply_common.h for the GEMM convention).
//
// Notation per element: d = D nodes and Q Gauss points per axis; reference-gradient
// channels at a quadrature point (a,b,c) are dx = G_x B_y B_z u, dy = B_x G_y B_z u,
// dz = B_x B_y G_z u and, when the mass term is present, the value u = B_x B_y B_z u.
//
// Each descriptor provides
//   NCOL       GEMM columns per element (the two untouched tensor indices),
//   C, NT      length of the contracted index and number of K-stacked input tensors,
//   O          output rows (the new 1-D index; 2Q when B and G rows are stacked),
//   in_off(t)  offset of input tensor t inside the element's input region,
//   A(tab,o,k) the stacked pass matrix (k = t*C + c),
//   out(o,n)   element-local output address, or -1 to drop the row/column pair.
#pragma once
#include "apply_common.h"

namespace hexpa {

// ======================================================================== diffusion
// Forward stage x: X[n=(j,k)][i] -> U1[o1][n], rows o1 < Q: B, o1 >= Q: G.
template <int D, int Q, bool M>
struct DF1 {
    static constexpr int NCOL = D * D, C = D, NT = 1, O = 2 * Q;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return o < Q ? tB(t, o, k, D) : tG(t, o - Q, k, D); }
    __device__ static int out(int o, int n) { return n + NCOL * o; }
};
// Forward stage y: U1[n=(k,o1)][j] -> U2[m(o1,o2)][k]; the (G,G) combinations are dropped:
// m = o1 + 2Q o2 for o2 < Q, and 2Q^2 + o1 + Q (o2 - Q) for o2 >= Q, o1 < Q.
template <int D, int Q, bool M>
struct DF2 {
    static constexpr int NCOL = 2 * Q * D, C = D, NT = 1, O = 2 * Q;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return o < Q ? tB(t, o, k, D) : tG(t, o - Q, k, D); }
    __device__ static int out(int o2, int n)
    {
        const int o1 = n / D, k = n - o1 * D;
        int m;
        if (o2 < Q)
            m = o1 + 2 * Q * o2;
        else if (o1 < Q)
            m = 2 * Q * Q + o1 + Q * (o2 - Q);
        else
            return -1;
        return k + D * m;
    }
};
// Forward stage z: U2[m][k] -> channels V[ch][c][b][a]; exactly one G among (o1,o2,o3)
// gives dx/dy/dz, none gives the value channel (kept only with the mass term).
template <int D, int Q, bool M>
struct DF3 {
    static constexpr int NCOL = 3 * Q * Q, C = D, NT = 1, O = 2 * Q;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return o < Q ? tB(t, o, k, D) : tG(t, o - Q, k, D); }
    __device__ static int out(int o3, int m)
    {
        int o1, o2;
        if (m < 2 * Q * Q) {
            o2 = m / (2 * Q);
            o1 = m - o2 * 2 * Q;
        } else {
            const int mm = m - 2 * Q * Q;
            const int r = mm / Q;
            o1 = mm - r * Q;
            o2 = Q + r;
        }
        const int gx = o1 >= Q, gy = o2 >= Q, gz = o3 >= Q;
        const int a = o1 - gx * Q, b = o2 - gy * Q, c = o3 - gz * Q;
        int ch;
        if (gx + gy + gz == 1)
            ch = gx ? 0 : (gy ? 1 : 2);
        else if (gx + gy + gz == 0 && M)
            ch = 3;
        else
            return -1;
        return ch * Q * Q * Q + a + Q * (b + Q * c);
    }
};
// Transposed stage x, channel dx: V0[n=(b,c)][a] -> W0[i][n] with G^T.
template <int D, int Q, bool M>
struct DT1a {
    static constexpr int NCOL = Q * Q, C = Q, NT = 1, O = D;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tG(t, k, o, D); }
    __device__ static int out(int o, int n) { return n + Q * Q * o; }
};
// Transposed stage x, channels dy, dz (and value): B^T; W_ch[i][n] at ch*Q*Q*D.
template <int D, int Q, bool M>
struct DT1b {
    static constexpr int NCH = M ? 3 : 2;
    static constexpr int NCOL = NCH * Q * Q, C = Q, NT = 1, O = D;
    __device__ static int in_off(int) { return Q * Q * Q; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, D); }
    __device__ static int out(int o, int n)
    {
        const int ch = 1 + n / (Q * Q), nn = n - (ch - 1) * Q * Q;
        return ch * Q * Q * D + nn + Q * Q * o;
    }
};
// Transposed stage y, path continuing with B_z^T: t1 = B_y^T W0 + G_y^T W1 (+ B_y^T W3).
template <int D, int Q, bool M>
struct DT2a {
    static constexpr int NCOL = Q * D, C = Q, NT = M ? 3 : 2, O = D;
    __device__ static int in_off(int t) { return (t == 2 ? 3 : t) * Q * Q * D; }
    __device__ static double A(const DevTables *tb, int o, int k)
    {
        const int t = k / Q, b = k - t * Q;
        return t == 1 ? tG(tb, b, o, D) : tB(tb, b, o, D);
    }
    __device__ static int out(int o, int n) { return n + Q * D * o; }
};
// Transposed stage y, path continuing with G_z^T: t2 = B_y^T W2.
template <int D, int Q, bool M>
struct DT2b {
    static constexpr int NCOL = Q * D, C = Q, NT = 1, O = D;
    __device__ static int in_off(int) { return 2 * Q * Q * D; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, D); }
    __device__ static int out(int o, int n) { return D * D * Q + n + Q * D * o; }
};
// Transposed stage z: y_E[k][n=(i,j)] = B_z^T t1 + G_z^T t2 (K-stacked), scattered to y.
template <int D, int Q, bool M>
struct DT3 {
    static constexpr int NCOL = D * D, C = Q, NT = 2, O = D;
    __device__ static int in_off(int t) { return t * Q * D * D; }
    __device__ static double A(const DevTables *tb, int o, int k)
    {
        const int t = k / Q, c = k - t * Q;
        return t == 0 ? tB(tb, c, o, D) : tG(tb, c, o, D);
    }
    __device__ static int out(int o, int n) { return n + D * D * o; }
};

// ======================================================================== mass
template <int D, int Q>
struct MF1 {
    static constexpr int NCOL = D * D, C = D, NT = 1, O = Q;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, D); }
    __device__ static int out(int o, int n) { return n + NCOL * o; }
};
template <int D, int Q>
struct MF2 {
    static constexpr int NCOL = Q * D, C = D, NT = 1, O = Q;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, D); }
    __device__ static int out(int o, int n) { return n + NCOL * o; }
};
template <int D, int Q>
struct MF3 {
    static constexpr int NCOL = Q * Q, C = D, NT = 1, O = Q;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, o, k, D); }
    __device__ static int out(int o, int n) { return n + NCOL * o; }
};
template <int D, int Q>
struct MT1 {
    static constexpr int NCOL = Q * Q, C = Q, NT = 1, O = D;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, D); }
    __device__ static int out(int o, int n) { return n + NCOL * o; }
};
template <int D, int Q>
struct MT2 {
    static constexpr int NCOL = Q * D, C = Q, NT = 1, O = D;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, D); }
    __device__ static int out(int o, int n) { return n + NCOL * o; }
};
template <int D, int Q>
struct MT3 {
    static constexpr int NCOL = D * D, C = Q, NT = 1, O = D;
    __device__ static int in_off(int) { return 0; }
    __device__ static double A(const DevTables *t, int o, int k) { return tB(t, k, o, D); }
    __device__ static int out(int o, int n) { return n + NCOL * o; }
};

}  // namespace hexpa
