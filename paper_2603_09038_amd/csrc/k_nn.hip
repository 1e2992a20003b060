// Kernels of the learned preconditioner: the per-element 3-layer convolutional network
// on the (p+1)^3 nodal tile (3x3x3 cross-correlation, zero padding 1, bias, ReLU between
// layers), its backward pass and Adam, the tile gather/normalisation and the averaged
// scatter of the element outputs, and the p=1 coarse level of the two-level preconditioner.
//
// Activations are stored [element][channel][point], point = i + N j + N^2 k (the
// operator's local node order); weights are [c_out][c_in][tap], tap = tx + 3 ty + 9 tz
// reading the neighbour (i + tx - 1, j + ty - 1, k + tz - 1).  Work tiles sit in LDS with
// a guard band on both sides so every shifted read is in bounds; reads that fall outside
// the element are multiplied by 0 (zero padding).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "k_nn.h"

namespace hexpa {

namespace {

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <int N>
struct Tile {
    static constexpr int P = N * N * N;
    static constexpr int GUARD = 1 + N + N * N;  // largest |offset| of a 3x3x3 neighbour
    // elements per workgroup and workgroup size (a multiple of the wave size)
    static constexpr int EPB = N == 3 ? 4 : (N == 4 ? 4 : 2);
    static constexpr int THREADS = ((EPB * P + 63) / 64) * 64;
    __host__ __device__ static constexpr int off(int tap)
    {
        return (tap % 3 - 1) + N * ((tap / 3) % 3 - 1) + N * N * (tap / 9 - 1);
    }
};

// 0/1 factors of the 27 neighbours of point pt (1 inside the tile).
template <int N>
__device__ inline void tap_mask(int pt, float (&mk)[27])
{
    const int i = pt % N, j = (pt / N) % N, k = pt / (N * N);
    const float mx[3] = {i > 0 ? 1.f : 0.f, 1.f, i < N - 1 ? 1.f : 0.f};
    const float my[3] = {j > 0 ? 1.f : 0.f, 1.f, j < N - 1 ? 1.f : 0.f};
    const float mz[3] = {k > 0 ? 1.f : 0.f, 1.f, k < N - 1 ? 1.f : 0.f};
#pragma unroll
    for (int t = 0; t < 27; ++t) mk[t] = mx[t % 3] * my[(t / 3) % 3] * mz[t / 9];
}

// out[e][o][pt] = bias[o] + sum_c sum_tap Wt[c][tap][o] in[e][c][pt + off(tap)]  (zero padded),
// then ReLU (RELU) or a multiply by [a_mask > 0] (MASK, the backward of a ReLU).
// Wt is the weight tensor already transposed to [c][tap][o]; bias may be null.
template <int N, int CIN, int COUT, bool RELU, bool MASK>
__global__ __launch_bounds__(Tile<N>::THREADS) void k_conv(int64_t nelem, const float *__restrict__ in,
                                                           const float *__restrict__ Wt,
                                                           const float *__restrict__ bias,
                                                           const float *__restrict__ a_mask, float *__restrict__ out)
{
    using T = Tile<N>;
    constexpr int NW = CIN * 27 * COUT, NX = T::EPB * CIN * T::P;
    __shared__ float sw[NW];
    __shared__ float sx[T::GUARD + NX + T::GUARD];
    const int t = threadIdx.x;
    const int64_t e0 = (int64_t)blockIdx.x * T::EPB;
    const int64_t nin = std::min((int64_t)T::EPB, nelem - e0) * CIN * T::P;
    for (int i = t; i < NW; i += T::THREADS) sw[i] = Wt[i];
    for (int i = t; i < T::GUARD; i += T::THREADS) sx[i] = sx[T::GUARD + NX + i] = 0.f;
    for (int i = t; i < NX; i += T::THREADS) sx[T::GUARD + i] = i < nin ? in[e0 * CIN * T::P + i] : 0.f;
    __syncthreads();
    const int el = t / T::P, pt = t % T::P;
    if (el >= T::EPB || e0 + el >= nelem) return;
    float mk[27];
    tap_mask<N>(pt, mk);
    float acc[COUT];
#pragma unroll
    for (int o = 0; o < COUT; ++o) acc[o] = bias ? bias[o] : 0.f;
    const float *xs = sx + T::GUARD + el * CIN * T::P + pt;
#pragma unroll 1
    for (int c = 0; c < CIN; ++c) {
        const float *xc = xs + c * T::P;
        const float *wc = sw + c * 27 * COUT;
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) {
            const float v = xc[T::off(tap)] * mk[tap];
#pragma unroll
            for (int o = 0; o < COUT; ++o) acc[o] = fmaf(wc[tap * COUT + o], v, acc[o]);
        }
    }
    const int64_t ob = (e0 + el) * COUT * T::P + pt;
#pragma unroll
    for (int o = 0; o < COUT; ++o) {
        float v = acc[o];
        if (RELU) v = fmaxf(v, 0.f);
        if (MASK) v = a_mask[ob + o * T::P] > 0.f ? v : 0.f;
        out[ob + o * T::P] = v;
    }
}

// Wt[c][tap][o] = W[o][c][tap] (forward) or, for the input gradient, the flipped
// adjoint Wt[o][tap][c] = W[o][c][26 - tap] read as a (COUT -> CIN) convolution.
__global__ void k_transpose_w(const float *__restrict__ W, int cout, int cin, int adjoint, float *__restrict__ Wt)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= cout * cin * 27) return;
    const int tap = i % 27, c = (i / 27) % cin, o = i / (27 * cin);
    if (!adjoint) Wt[(c * 27 + tap) * cout + o] = W[i];
    else Wt[(o * 27 + (26 - tap)) * cin + c] = W[i];
}

// Weight/bias gradient partial sums: dW[o][c][tap] = sum_e sum_pt dout[e][o][pt] in[e][c][pt + off(tap)],
// db[o] = sum dout.  Thread = (c, group of OB outputs, slice of points); workgroup g
// handles elements g, g + G, ...; row (g, slice) of `partial` receives the thread sums.
template <int CIN, int COUT>
struct WgradShape {
    static constexpr int OB = COUT >= 4 ? 4 : 1;
    static constexpr int NPAIR = CIN * (COUT / OB);
    static constexpr int SL = 256 / NPAIR;
    static constexpr int NT = COUT * CIN * 27 + COUT;
    static_assert(COUT % OB == 0 && NPAIR <= 256 && 256 % NPAIR == 0, "thread layout");
};
constexpr int kWgradBlocks = 768;  // three workgroups per CU: the 16x16 layer's 162 registers allow three

template <int N, int CIN, int COUT>
__global__ __launch_bounds__(256) void k_conv_wgrad(int64_t nelem, const float *__restrict__ in,
                                                    const float *__restrict__ dout, float *__restrict__ partial)
{
    using T = Tile<N>;
    using S = WgradShape<CIN, COUT>;
    constexpr int OB = S::OB, NX = CIN * T::P;
    __shared__ float sx[T::GUARD + NX + T::GUARD];
    __shared__ float sd[COUT * T::P];
    const int t = threadIdx.x;
    const int pair = t % S::NPAIR, sl = t / S::NPAIR;
    const int c = pair % CIN, og = pair / CIN;
    float acc[OB][27], bacc[OB];
#pragma unroll
    for (int u = 0; u < OB; ++u) {
        bacc[u] = 0.f;
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) acc[u][tap] = 0.f;
    }
    for (int i = t; i < T::GUARD; i += 256) sx[i] = sx[T::GUARD + NX + i] = 0.f;
    for (int64_t e = blockIdx.x; e < nelem; e += gridDim.x) {
        __syncthreads();
        for (int i = t; i < NX; i += 256) sx[T::GUARD + i] = in[e * NX + i];
        for (int i = t; i < COUT * T::P; i += 256) sd[i] = dout[e * COUT * T::P + i];
        __syncthreads();
        for (int pt = sl; pt < T::P; pt += S::SL) {
            float mk[27];
            tap_mask<N>(pt, mk);
            float g[OB];
#pragma unroll
            for (int u = 0; u < OB; ++u) {
                g[u] = sd[(og * OB + u) * T::P + pt];
                bacc[u] += g[u];
            }
            const float *xc = sx + T::GUARD + c * T::P + pt;
#pragma unroll
            for (int tap = 0; tap < 27; ++tap) {
                const float v = xc[T::off(tap)] * mk[tap];
#pragma unroll
                for (int u = 0; u < OB; ++u) acc[u][tap] = fmaf(g[u], v, acc[u][tap]);
            }
        }
    }
    float *row = partial + ((int64_t)blockIdx.x * S::SL + sl) * S::NT;
#pragma unroll
    for (int u = 0; u < OB; ++u) {
        const int o = og * OB + u;
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) row[(o * CIN + c) * 27 + tap] = acc[u][tap];
        if (c == 0) row[COUT * CIN * 27 + o] = bacc[u];
    }
}

// grad[w] += sum over rows of partial[row][w] in two passes, each in a fixed order (FP64
// accumulation, so the result is reproducible): the rows are cut into kReduceChunks chunks;
// a workgroup takes 64 columns of one chunk, its four waves summing every fourth row of it
// and their four sums added in wave order (part2[chunk][w], FP64); then one thread per
// column adds the chunks in order.  (One thread per column over all rows left most of the
// GPU idle: a layer has 433-6928 weights, so 2-28 workgroups.)
constexpr int kReduceChunks = 64;

__global__ __launch_bounds__(256) void k_reduce_chunks(const float *__restrict__ partial, int rows, int nt,
                                                       double *__restrict__ part2)
{
    __shared__ double red[4][64];
    const int l = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int w = blockIdx.x * 64 + l, chunk = blockIdx.y;
    const int r0 = (int)((int64_t)rows * chunk / kReduceChunks);
    const int r1 = (int)((int64_t)rows * (chunk + 1) / kReduceChunks);
    double a = 0.0;
    if (w < nt)
        for (int g = r0 + sl; g < r1; g += 4) a += partial[(int64_t)g * nt + w];
    red[sl][l] = a;
    __syncthreads();
    if (sl == 0 && w < nt) part2[(int64_t)chunk * nt + w] = ((red[0][l] + red[1][l]) + red[2][l]) + red[3][l];
}

__global__ void k_reduce_rows(const double *__restrict__ part2, int nt, float *__restrict__ grad)
{
    const int w = blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nt) return;
    double a = 0.0;
    for (int c = 0; c < kReduceChunks; ++c) a += part2[(int64_t)c * nt + w];
    grad[w] += (float)a;
}

template <int N>
__global__ __launch_bounds__(128) void k_nn_input(int64_t nelem, const double *__restrict__ r,
                                                  const int32_t *__restrict__ emap, const float *__restrict__ logk,
                                                  float *__restrict__ x0, float *__restrict__ s_out)
{
    constexpr int P = N * N * N;
    static_assert(P <= 128, "one point per thread");
    __shared__ double red[128];
    const int64_t e = blockIdx.x;
    const int t = threadIdx.x;
    const double v = t < P ? r[emap[e * P + t]] : 0.0;
    red[t] = v * v;
    __syncthreads();
    for (int h = 64; h > 0; h >>= 1) {
        if (t < h) red[t] += red[t + h];
        __syncthreads();
    }
    const double rms = sqrt(red[0] / P);
    const double s = rms > 0.0 ? rms : 1.0;
    if (t < P) {
        const float xv = (float)(v / s), lk = logk[e * P + t];
        x0[(e * 2 + 0) * P + t] = xv;  // tile e: +r
        x0[(e * 2 + 1) * P + t] = lk;
        x0[((nelem + e) * 2 + 0) * P + t] = -xv;  // tile nelem + e: -r
        x0[((nelem + e) * 2 + 1) * P + t] = lk;
    }
    if (t == 0) s_out[e] = (float)s;
}

// z[g] += s_e (out(+r)_e - out(-r)_e) / 2 * inv_mult[g]: the odd part of the network,
// averaged over the elements sharing g.  out holds the +r tiles, then the -r tiles.
__global__ void k_nn_output(int64_t total, int P, const float *__restrict__ out, const float *__restrict__ s,
                            const int32_t *__restrict__ emap, const double *__restrict__ inv_mult, double scale,
                            double *__restrict__ z)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int g = emap[idx];
    const double odd = 0.5 * scale * ((double)out[idx] - (double)out[total + idx]);
    unsafeAtomicAdd(z + g, odd * (double)s[idx / P] * inv_mult[g]);
}

// adjoint: d/d out(+r) = s_e gz inv_mult / 2, d/d out(-r) = its negative
__global__ void k_nn_output_grad(int64_t total, int P, const double *__restrict__ gz, const float *__restrict__ s,
                                 const int32_t *__restrict__ emap, const double *__restrict__ inv_mult,
                                 float *__restrict__ gout)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= total) return;
    const int g = emap[idx];
    const float v = (float)(0.5 * gz[g] * inv_mult[g] * (double)s[idx / P]);
    gout[idx] = v;
    gout[total + idx] = -v;
}

__global__ void k_count(int64_t total, const int32_t *__restrict__ emap, double *__restrict__ cnt)
{
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < total) unsafeAtomicAdd(cnt + emap[idx], 1.0);
}
__global__ void k_recip_or_zero(int64_t n, double *__restrict__ v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = v[i] > 0.0 ? 1.0 / v[i] : 0.0;
}
__global__ void k_fill_f32(float *y, float v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = v;
}

__global__ void k_adam(float *__restrict__ p, float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int n, float lr, float bc1, float bc2)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / bc1) / (sqrtf(vi / bc2) + eps);
    g[i] = 0.0f;
}

__global__ void k_sub(double *y, const double *a, const double *b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a[i] - b[i];
}
__global__ void k_mul(double *y, const double *a, const double *b, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = a[i] * b[i];
}

__global__ void k_loss_scale(double *g, int64_t n, double *sc)
{
    const double den = sc[1];
    const double f = den > 0.0 ? 2.0 / den : 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        g[i] *= f;
    if (blockIdx.x == 0 && threadIdx.x == 0) sc[2] = den > 0.0 ? sc[0] / den : 0.0;
}

// ---------------------------------------------------------------- coarse level
// 1-D weight of coarse vertex a at fine lattice index I: the fine node lies in element
// ex = min(I / p, n - 1) at GLL coordinate xi = gll[I - ex p]; the p=1 basis there is
// (1 - xi) at vertex ex and xi at vertex ex + 1.
__device__ inline double w1d(int64_t I, int64_t a, int n, int p, const double *gll)
{
    const int64_t ex = min(I / p, (int64_t)n - 1);
    const double xi = gll[I - ex * p];
    return a == ex ? 1.0 - xi : (a == ex + 1 ? xi : 0.0);
}

__global__ void k_prolong(BoxDims b, const double *__restrict__ gll, const double *__restrict__ u1,
                          double *__restrict__ uf, int add)
{
    const int64_t Mx = (int64_t)b.nx * b.p + 1, My = (int64_t)b.ny * b.p + 1, Mz = (int64_t)b.nz * b.p + 1;
    const int64_t Cx = b.nx + 1, Cy = b.ny + 1;
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= Mx * My * Mz) return;
    const int64_t I = g % Mx, J = (g / Mx) % My, K = g / (Mx * My);
    const int64_t ex = min(I / b.p, (int64_t)b.nx - 1), ey = min(J / b.p, (int64_t)b.ny - 1),
                  ez = min(K / b.p, (int64_t)b.nz - 1);
    const double x = gll[I - ex * b.p], y = gll[J - ey * b.p], z = gll[K - ez * b.p];
    double v = 0.0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int ca = c & 1, cb = (c >> 1) & 1, cc = c >> 2;
        const double w = (ca ? x : 1.0 - x) * (cb ? y : 1.0 - y) * (cc ? z : 1.0 - z);
        v += w * u1[(ex + ca) + Cx * ((ey + cb) + Cy * (ez + cc))];
    }
    uf[g] = add ? uf[g] + v : v;
}

// Restriction r1 = P1^T rf, separable: the weight of fine node (I,J,K) at coarse vertex
// (a,b,c) is w(I,a) w(J,b) w(K,c), so three 1-D passes (x, then y, then z), each summing
// the at most 2p + 1 fine lattice points whose 1-D weight for a coarse index is nonzero,
// in a fixed order (no atomics).  Pass `axis` maps in[nz'][ny'][nx'] to out with that
// axis shortened from M = n p + 1 to n + 1.
__global__ void k_restrict_axis(int axis, int n, int p, int64_t nx_in, int64_t ny_in, int64_t nz_in,
                                const double *__restrict__ gll, const double *__restrict__ in,
                                double *__restrict__ out)
{
    const int64_t C = n + 1, M = (int64_t)n * p + 1;
    const int64_t ox = axis == 0 ? C : nx_in, oy = axis == 1 ? C : ny_in, oz = axis == 2 ? C : nz_in;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= ox * oy * oz) return;
    const int64_t i = idx % ox, j = (idx / ox) % oy, k = idx / (ox * oy);
    const int64_t a = axis == 0 ? i : (axis == 1 ? j : k);  // coarse index along the axis
    const int64_t stride = axis == 0 ? 1 : (axis == 1 ? nx_in : nx_in * ny_in);
    const int64_t base = (axis == 0 ? 0 : i) + nx_in * ((axis == 1 ? 0 : j) + ny_in * (axis == 2 ? 0 : k));
    const int64_t I0 = max((int64_t)0, (a - 1) * p), I1 = min(M - 1, (a + 1) * p);
    double acc = 0.0;
    for (int64_t I = I0; I <= I1; ++I) {
        const double w = w1d(I, a, n, p, gll);
        if (w != 0.0) acc = fma(w, in[base + I * stride], acc);
    }
    out[idx] = acc;
}

__global__ void k_probe_vec(BoxDims b, int cls, double *__restrict__ v)
{
    const int64_t Cx = b.nx + 1, Cy = b.ny + 1, Cz = b.nz + 1;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= Cx * Cy * Cz) return;
    const int64_t I = i % Cx, J = (i / Cx) % Cy, K = i / (Cx * Cy);
    v[i] = (I % 3 == cls % 3 && J % 3 == (cls / 3) % 3 && K % 3 == cls / 9) ? 1.0 : 0.0;
}

// Within the 3x3x3 neighbourhood of vertex i exactly one vertex has class cls; the entry
// of A v_cls at i is therefore A[i][j] for that neighbour j (0 if j is off the lattice).
// S is stored [slot][i], slot = (dx+1) + 3 (dy+1) + 9 (dz+1).  Constrained rows and
// columns (ess) become those of the identity.
__global__ void k_probe_gather(BoxDims b, int cls, const double *__restrict__ y, const uint8_t *__restrict__ ess,
                               double *__restrict__ S)
{
    const int64_t Cx = b.nx + 1, Cy = b.ny + 1, Cz = b.nz + 1, n1 = Cx * Cy * Cz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n1) return;
    const int64_t I = i % Cx, J = (i / Cx) % Cy, K = i / (Cx * Cy);
    auto delta = [](int64_t X, int want) {
        const int d = (int)(((want - X) % 3 + 3) % 3);
        return d == 2 ? -1 : d;
    };
    const int dx = delta(I, cls % 3), dy = delta(J, (cls / 3) % 3), dz = delta(K, cls / 9);
    const int slot = (dx + 1) + 3 * (dy + 1) + 9 * (dz + 1);
    const int64_t In = I + dx, Jn = J + dy, Kn = K + dz;
    double v = 0.0;
    if (In >= 0 && In < Cx && Jn >= 0 && Jn < Cy && Kn >= 0 && Kn < Cz) {
        const int64_t j = In + Cx * (Jn + Cy * Kn);
        v = y[i];
        if (ess && (ess[i] || ess[j])) v = (j == i && ess[i]) ? 1.0 : 0.0;
    }
    S[slot * n1 + i] = v;
}

__global__ void k_dinv_center(int64_t n1, const double *__restrict__ S, double *__restrict__ dinv)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n1) dinv[i] = 1.0 / S[13 * n1 + i];
}

// Block sum in a fixed order; the last workgroup to finish adds the per-block partials in
// block order and hands the total to fin (thread 0 only), then re-arms the counter.
// Blocks of kCoarseThreads threads (small blocks spread the 27-point stencil over more CUs).
constexpr int kCoarseThreads = 256;
template <class F>
__device__ inline void grid_sum_last(double v, double *partial, unsigned int *count, F fin)
{
    __shared__ double sh[kCoarseThreads];
    __shared__ int last;
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int h = kCoarseThreads / 2; h > 0; h >>= 1) {
        if (t < h) sh[t] += sh[t + h];
        __syncthreads();
    }
    if (t == 0) {
        partial[blockIdx.x] = sh[0];
        __threadfence();
        const unsigned prev = atomicAdd(count, 1u);
        last = prev == gridDim.x - 1;
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double a = 0.0;
    for (int i = t; i < (int)gridDim.x; i += kCoarseThreads)
        a += __hip_atomic_load(partial + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sh[t] = a;
    __syncthreads();
    for (int h = kCoarseThreads / 2; h > 0; h >>= 1) {
        if (t < h) sh[t] += sh[t + h];
        __syncthreads();
    }
    if (t == 0) {
        fin(sh[0]);
        __hip_atomic_store(count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// u = 0, z = dinv r, p0 = 0; rz = r.z, beta = 0
__global__ __launch_bounds__(kCoarseThreads) void k_cpcg_init(int64_t n1, const double *__restrict__ dinv,
                                                   const double *__restrict__ r, double *__restrict__ u,
                                                   double *__restrict__ z, double *__restrict__ p0, double *partial,
                                                   CoarseScalars *sc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (i < n1) {
        const double zi = dinv[i] * r[i];
        z[i] = zi;
        u[i] = 0.0;
        p0[i] = 0.0;
        v = r[i] * zi;
    }
    grid_sum_last(v, partial, &sc->count, [&](double tot) {
        sc->rz = tot;
        sc->beta = 0.0;
    });
}

// p1 = z + beta p0; Ap = S (z + beta p0); alpha = rz / (p1 . Ap)
__global__ __launch_bounds__(kCoarseThreads) void k_cpcg_a(BoxDims b, const double *__restrict__ S,
                                                const double *__restrict__ z, const double *__restrict__ p0,
                                                double *__restrict__ p1, double *__restrict__ Ap, double *partial,
                                                CoarseScalars *sc)
{
    const int64_t Cx = b.nx + 1, Cy = b.ny + 1, Cz = b.nz + 1, n1 = Cx * Cy * Cz;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double beta = sc->beta;
    double v = 0.0;
    if (i < n1) {
        const int64_t I = i % Cx, J = (i / Cx) % Cy, K = i / (Cx * Cy);
        double acc = 0.0;
#pragma unroll
        for (int s = 0; s < 27; ++s) {
            const int dx = s % 3 - 1, dy = (s / 3) % 3 - 1, dz = s / 9 - 1;
            const int64_t In = I + dx, Jn = J + dy, Kn = K + dz;
            if (In < 0 || In >= Cx || Jn < 0 || Jn >= Cy || Kn < 0 || Kn >= Cz) continue;
            const int64_t j = i + dx + Cx * (dy + Cy * dz);
            acc = fma(S[s * n1 + i], z[j] + beta * p0[j], acc);
        }
        const double pi = z[i] + beta * p0[i];
        p1[i] = pi;
        Ap[i] = acc;
        v = pi * acc;
    }
    grid_sum_last(v, partial, &sc->count, [&](double tot) {
        sc->pAp = tot;
        sc->alpha = tot > 0.0 ? sc->rz / tot : 0.0;
    });
}

// u += alpha p1; r -= alpha Ap; z = dinv r; beta = (r.z)_new / rz
__global__ __launch_bounds__(kCoarseThreads) void k_cpcg_b(int64_t n1, const double *__restrict__ dinv,
                                                const double *__restrict__ p1, const double *__restrict__ Ap,
                                                double *__restrict__ u, double *__restrict__ r,
                                                double *__restrict__ z, double *partial, CoarseScalars *sc)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const double alpha = sc->alpha;
    double v = 0.0;
    if (i < n1) {
        u[i] = fma(alpha, p1[i], u[i]);
        const double ri = fma(-alpha, Ap[i], r[i]);
        r[i] = ri;
        const double zi = dinv[i] * ri;
        z[i] = zi;
        v = ri * zi;
    }
    grid_sum_last(v, partial, &sc->count, [&](double tot) {
        sc->beta = sc->rz > 0.0 ? tot / sc->rz : 0.0;
        sc->rz = tot;
    });
}

// ---------------------------------------------------------------- FP16 MFMA inference
// The whole network part z += W G^T (s_e NN(G_e r / s_e, log kappa_e)) for one element per
// workgroup: gather and RMS-normalise the residual tile, three convolutions as implicit
// GEMMs on v_mfma_f32_16x16x16f16 (FP16 operands, FP32 accumulation), and the averaged
// scatter.  Layers 1 and 2 compute Y^T = W^T X^T: GEMM rows are the 16 output channels,
// columns 16 tile points (one row tile of the tile), and one k-step of 16 is one tap's 16
// input channels (layer 1: four taps of the two input channels padded to four).  Lane
// layout (pinned by the 16-bit lane-layout test): A lane l holds A[l%16][4(l/16)+t], B
// lane l holds B[4(l/16)+t][l%16], result lane l element v is D[4(l/16)+v][l%16], so a
// lane reads and writes four consecutive channels of one point.  Activations live in LDS
// as [padded point][channel] FP16 on the (N+2)^3 grid with a zero halo, so every shifted
// operand read is one 8-byte load.  Layer 3 (16 -> 1) is Y[pt][tap] = sum_c a2[pt][c]
// W3[c][tap] on MFMA followed by out[pt] = b3 + sum_tap Y[pt + off(tap)][tap] over the taps
// that stay in the tile.
typedef _Float16 h4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
constexpr int kPackL1 = 7, kPackL2 = 27, kPackL3 = 2, kPackSteps = kPackL1 + kPackL2 + kPackL3;

// Weight tables in lane order: step s, lane l -> 4 halves, entry (k = 4(l/16)+t, output
// channel l%16): the A-operand of layers 1-2 (row = output channel) and the B-operand of
// layer 3 (column = tap).
__global__ void k_pack16(const float *__restrict__ prm, h4_t *__restrict__ wp)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= kPackSteps * 64) return;
    const int s = i / 64, l = i % 64, g = l >> 4, col = l & 15;
    h4_t w;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        float v = 0.f;
        if (s < kPackL1) {  // rows = (tap 4s+g, channel t): W1[o][t][tap], channels 2, 3 zero
            const int tap = 4 * s + g;
            if (t < kNetCin && tap < 27) v = prm[kNetOffW1 + (col * kNetCin + t) * 27 + tap];
        } else if (s < kPackL1 + kPackL2) {  // rows = channel 4g+t of tap s-7: W2[o][c][tap]
            const int tap = s - kPackL1, c = 4 * g + t;
            v = prm[kNetOffW2 + (col * kNetCh + c) * 27 + tap];
        } else {  // rows = channel 4g+t, columns = taps 16 ct + col: W3[0][c][tap]
            const int ct = s - kPackL1 - kPackL2, c = 4 * g + t, tap = 16 * ct + col;
            if (tap < 27) v = prm[kNetOffW3 + c * 27 + tap];
        }
        w[t] = (_Float16)v;
    }
    wp[i] = w;
}

template <int N>
struct Pad {
    static constexpr int P = N * N * N, NP = N + 2, NP3 = NP * NP * NP, RT = (P + 15) / 16;
    __host__ __device__ static constexpr int off(int tap)
    {
        return (tap % 3 - 1) + NP * ((tap / 3) % 3 - 1) + NP * NP * (tap / 9 - 1);
    }
    __device__ static int pad(int pt)
    {
        const int i = pt % N, j = (pt / N) % N, k = pt / (N * N);
        return (i + 1) + NP * ((j + 1) + NP * (k + 1));
    }
    __device__ static bool halo(int q)
    {
        const int i = q % NP, j = (q / NP) % NP, k = q / (NP * NP);
        return i == 0 || j == 0 || k == 0 || i == NP - 1 || j == NP - 1 || k == NP - 1;
    }
};

template <int N>
__global__ __launch_bounds__(256, 2) void k_net16(int64_t nelem, const double *__restrict__ r,
                                                  const int32_t *__restrict__ emap, const float *__restrict__ logk,
                                                  const h4_t *__restrict__ wp, const float *__restrict__ prm,
                                                  const double *__restrict__ inv_mult, double scale,
                                                  double *__restrict__ z)
{
    // One element per workgroup of four waves: wave w owns GEMM row tiles w, w + 4, ...
    // (16 tile points each), so each wave keeps few operands in flight and several
    // workgroups share a CU.  Every tile point belongs to one thread in the gather,
    // normalisation, layer-3 tap sum and scatter (P <= 256).  The layer-3 table is stored
    // tap-major with an odd row pitch (in 4-byte words), so the 27 shifted reads of a wave
    // hit distinct LDS banks.
    using T = Pad<N>;
    constexpr int P = T::P, NP3 = T::NP3, RT = T::RT;
    constexpr int YP = 16 * RT + 2;  // row pitch of the layer-3 table (halves; odd in words)
    static_assert(P <= 256, "one tile point per thread");
    __shared__ h4_t x0b[NP3];      // [point] (r/s, log kappa, 0, 0)
    __shared__ h4_t a1b[NP3 * 4];  // [point][channel group of 4]
    __shared__ h4_t a2b[NP3 * 4];
    __shared__ _Float16 yb[32 * YP];  // layer-3 table [tap][row]
    __shared__ double red[4];
    const int tid = threadIdx.x, l = tid & 63, g = l >> 4, col = l & 15;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const h4_t zero4 = {0, 0, 0, 0};
    for (int i = tid; i < NP3; i += 256) {
        x0b[i] = zero4;
#pragma unroll
        for (int k = 0; k < 4; ++k) a1b[i * 4 + k] = a2b[i * 4 + k] = zero4;
    }
    h4_t w1[kPackL1], w2[kPackL2], w3[kPackL3];
#pragma unroll
    for (int s = 0; s < kPackL1; ++s) w1[s] = wp[s * 64 + l];
#pragma unroll
    for (int s = 0; s < kPackL2; ++s) w2[s] = wp[(kPackL1 + s) * 64 + l];
#pragma unroll
    for (int s = 0; s < kPackL3; ++s) w3[s] = wp[(kPackL1 + kPackL2 + s) * 64 + l];
    // Layers 1 and 2 run transposed (D^T = W^T X^T: the packed weights as the A-operand, the
    // activations as the B-operand), so each lane ends with four consecutive output
    // channels 4g..4g+3 of one tile point and stores them with one 8-byte write.
    float bias1[4], bias2[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        bias1[v] = prm[kNetOffB1 + 4 * g + v];
        bias2[v] = prm[kNetOffB2 + 4 * g + v];
    }
    const float bias3 = prm[kNetOffB3];
    constexpr int MT = (RT + 3) / 4;  // row tiles per wave (the last ones may be absent)
    // A wave's tiles past RT (only when RT is not a multiple of 4) compute on clamped rows
    // and store nothing: the MFMA loops carry no per-tile branches.
    int rb[MT];                        // padded index of this lane's A-operand row (dummy rows repeat the last point)
    int op[MT];                        // padded index of the point whose channels this lane stores, -1 past the tile
    bool tv[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) {
        const int rt = wave + 4 * m;
        tv[m] = rt < RT;
        rb[m] = T::pad(min(16 * rt + col, P - 1));
        op[m] = (tv[m] && 16 * rt + col < P) ? rb[m] : -1;
    }
    int o1[kPackL1];  // layer-1 tap offset of this lane's k-group in every k-step (taps past 26: zero weights)
#pragma unroll
    for (int s = 0; s < kPackL1; ++s) o1[s] = 4 * s + g < 27 ? T::off(4 * s + g) : 0;
    const bool own = tid < P;  // this thread's tile point
    const int pp = own ? T::pad(tid) : 0;
    uint32_t inmask = 0;  // bit tap: the neighbour (tap) of this thread's point lies in the tile
    {
        const int pi = tid % N, pj = (tid / N) % N, pk = tid / (N * N);
#pragma unroll
        for (int tap = 0; tap < 27; ++tap) {
            const int dx = tap % 3 - 1, dy = (tap / 3) % 3 - 1, dz = tap / 9 - 1;
            if ((unsigned)(pi + dx) < (unsigned)N && (unsigned)(pj + dy) < (unsigned)N && (unsigned)(pk + dz) < (unsigned)N)
                inmask |= 1u << tap;
        }
    }
    __syncthreads();

    for (int64_t e = blockIdx.x; e < nelem; e += gridDim.x) {
        // gather r, element RMS
        int32_t gi = 0;
        double rv = 0.0;
        float lk = 0.f;
        if (own) {
            gi = emap[e * P + tid];
            rv = r[gi];
            lk = logk[e * P + tid];
        }
        double ss = rv * rv;
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) ss += __shfl_xor(ss, m);
        if (l == 0) red[wave] = ss;
        __syncthreads();
        ss = (red[0] + red[1]) + (red[2] + red[3]);
        const double rms = sqrt(ss / P);
        const double sc = rms > 0.0 ? rms : 1.0;

        // the network on +r and on -r; the preconditioner takes the odd part
        float odd = 0.f;
#pragma unroll 1
        for (int sgn = 0; sgn < 2; ++sgn) {
            if (own) {
                const h4_t v = {(_Float16)(float)((sgn ? -rv : rv) / sc), (_Float16)lk, (_Float16)0.f, (_Float16)0.f};
                x0b[pp] = v;
            }
            __syncthreads();
            f4_t acc[MT];
            // layer 1: 2 (padded to 4) -> 16 channels, ReLU
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m] = (f4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < kPackL1; ++s)
#pragma unroll
                for (int m = 0; m < MT; ++m)
                    acc[m] = __builtin_amdgcn_mfma_f32_16x16x16f16(w1[s], x0b[rb[m] + o1[s]], acc[m], 0, 0, 0);
#pragma unroll
            for (int m = 0; m < MT; ++m)
                if (op[m] >= 0) {
                    h4_t h;
#pragma unroll
                    for (int v = 0; v < 4; ++v) h[v] = (_Float16)fmaxf(acc[m][v] + bias1[v], 0.f);
                    a1b[op[m] * 4 + g] = h;
                }
            __syncthreads();
            // layer 2: 16 -> 16, one tap per k-step, ReLU; a compiler barrier before each tap
            // keeps the compiler from hoisting all 27 taps' operand loads (registers): measured
            // faster than chunks of 3, 9 or 27 taps
#pragma unroll
            for (int m = 0; m < MT; ++m) acc[m] = (f4_t){0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s0 = 0; s0 < 27; s0 += 1) {
                asm volatile("" ::: "memory");
#pragma unroll
                for (int s = s0; s < s0 + 1; ++s)
#pragma unroll
                    for (int m = 0; m < MT; ++m)
                        acc[m] = __builtin_amdgcn_mfma_f32_16x16x16f16(w2[s], a1b[(rb[m] + T::off(s)) * 4 + g],
                                                                       acc[m], 0, 0, 0);
            }
#pragma unroll
            for (int m = 0; m < MT; ++m)
                if (op[m] >= 0) {
                    h4_t h;
#pragma unroll
                    for (int v = 0; v < 4; ++v) h[v] = (_Float16)fmaxf(acc[m][v] + bias2[v], 0.f);
                    a2b[op[m] * 4 + g] = h;
                }
            __syncthreads();
            // layer 3, part 1: Y[pt][tap] for every tile point and tap (rows past the tile unused)
#pragma unroll
            for (int ct = 0; ct < kPackL3; ++ct)
#pragma unroll
                for (int m = 0; m < MT; ++m) {
                    const f4_t y = __builtin_amdgcn_mfma_f32_16x16x16f16(a2b[rb[m] * 4 + g], w3[ct],
                                                                         (f4_t){0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
                    if (tv[m])
#pragma unroll
                        for (int v = 0; v < 4; ++v)
                            yb[(16 * ct + col) * YP + 16 * (wave + 4 * m) + 4 * g + v] = (_Float16)y[v];
                }
            __syncthreads();
            // layer 3, part 2: shifted sum over taps (the bias cancels in the odd part)
            if (own) {
                float o = bias3;
#pragma unroll
                for (int tap = 0; tap < 27; ++tap) {
                    const bool in = (inmask >> tap) & 1u;
                    const float yv = (float)yb[tap * YP + (in ? tid + Tile<N>::off(tap) : tid)];
                    o = in ? o + yv : o;
                }
                odd += sgn ? -0.5f * o : 0.5f * o;
            }
            // the next writes of x0b, a1 and yb come after the barrier at the top of the
            // next evaluation (x0b) or after further barriers (a1, yb)
        }
        // averaged scatter
        if (own) unsafeAtomicAdd(z + gi, (double)odd * sc * scale * inv_mult[gi]);
    }
}

template <int N>
hipError_t forward_t(int64_t nelem, const float *params, float *wt, const float *x0, float *a1, float *a2,
                     float *out, hipStream_t s)
{
    using T = Tile<N>;
    const unsigned nb = (unsigned)((nelem + T::EPB - 1) / T::EPB);
    float *w1 = wt, *w2 = wt + kNetW1, *w3 = w2 + kNetW2;
    hipLaunchKernelGGL(k_transpose_w, dim3(nblk(kNetW1)), dim3(256), 0, s, params + kNetOffW1, kNetCh, kNetCin, 0, w1);
    hipLaunchKernelGGL(k_transpose_w, dim3(nblk(kNetW2)), dim3(256), 0, s, params + kNetOffW2, kNetCh, kNetCh, 0, w2);
    hipLaunchKernelGGL(k_transpose_w, dim3(nblk(kNetW3)), dim3(256), 0, s, params + kNetOffW3, 1, kNetCh, 0, w3);
    hipLaunchKernelGGL((k_conv<N, kNetCin, kNetCh, true, false>), dim3(nb), dim3(T::THREADS), 0, s, nelem, x0, w1,
                       params + kNetOffB1, nullptr, a1);
    hipLaunchKernelGGL((k_conv<N, kNetCh, kNetCh, true, false>), dim3(nb), dim3(T::THREADS), 0, s, nelem, a1, w2,
                       params + kNetOffB2, nullptr, a2);
    hipLaunchKernelGGL((k_conv<N, kNetCh, 1, false, false>), dim3(nb), dim3(T::THREADS), 0, s, nelem, a2, w3,
                       params + kNetOffB3, nullptr, out);
    return hipGetLastError();
}

// floats of the largest block of partial rows (even, so the FP64 chunk sums behind it are
// 8-byte aligned)
inline int64_t partial_rows_floats()
{
    using L1 = WgradShape<kNetCin, kNetCh>;
    using L2 = WgradShape<kNetCh, kNetCh>;
    using L3 = WgradShape<kNetCh, 1>;
    const int64_t n = (int64_t)kWgradBlocks * std::max({L1::SL * L1::NT, L2::SL * L2::NT, L3::SL * L3::NT});
    return (n + 1) & ~(int64_t)1;
}

// grad_w holds the layer's weights followed by its biases: the order of a partial row.
template <int N, int CIN, int COUT>
void wgrad_layer(int64_t nelem, const float *in, const float *dout, float *partial, float *grad_w, hipStream_t s)
{
    using S = WgradShape<CIN, COUT>;
    hipLaunchKernelGGL((k_conv_wgrad<N, CIN, COUT>), dim3(kWgradBlocks), dim3(256), 0, s, nelem, in, dout, partial);
    // the chunk sums go behind the largest partial-row block (nn_partial_floats)
    double *part2 = reinterpret_cast<double *>(partial + partial_rows_floats());
    hipLaunchKernelGGL(k_reduce_chunks, dim3((S::NT + 63) / 64, kReduceChunks), dim3(256), 0, s, partial,
                       kWgradBlocks * S::SL, S::NT, part2);
    hipLaunchKernelGGL(k_reduce_rows, dim3(nblk(S::NT)), dim3(256), 0, s, part2, S::NT, grad_w);
}

template <int N>
hipError_t backward_t(int64_t nelem, const float *params, const float *x0, const float *a1, const float *a2,
                      const float *gout, float *ga2, float *ga1, float *grads, float *wt, float *partial,
                      hipStream_t s)
{
    using T = Tile<N>;
    const unsigned nb = (unsigned)((nelem + T::EPB - 1) / T::EPB);
    // layer 3: weights, then the gradient w.r.t. a2 masked by the ReLU
    wgrad_layer<N, kNetCh, 1>(nelem, a2, gout, partial, grads + kNetOffW3, s);
    hipLaunchKernelGGL(k_transpose_w, dim3(nblk(kNetW3)), dim3(256), 0, s, params + kNetOffW3, 1, kNetCh, 1, wt);
    hipLaunchKernelGGL((k_conv<N, 1, kNetCh, false, true>), dim3(nb), dim3(T::THREADS), 0, s, nelem, gout, wt,
                       nullptr, a2, ga2);
    // layer 2
    wgrad_layer<N, kNetCh, kNetCh>(nelem, a1, ga2, partial, grads + kNetOffW2, s);
    hipLaunchKernelGGL(k_transpose_w, dim3(nblk(kNetW2)), dim3(256), 0, s, params + kNetOffW2, kNetCh, kNetCh, 1, wt);
    hipLaunchKernelGGL((k_conv<N, kNetCh, kNetCh, false, true>), dim3(nb), dim3(T::THREADS), 0, s, nelem, ga2, wt,
                       nullptr, a1, ga1);
    // layer 1 (the input needs no gradient)
    wgrad_layer<N, kNetCin, kNetCh>(nelem, x0, ga1, partial, grads + kNetOffW1, s);
    return hipGetLastError();
}

}  // namespace

int64_t nn_partial_floats()
{
    using L1 = WgradShape<kNetCin, kNetCh>;
    using L2 = WgradShape<kNetCh, kNetCh>;
    using L3 = WgradShape<kNetCh, 1>;
    // partial rows, then the FP64 chunk sums (two floats each)
    return partial_rows_floats() + 2 * (int64_t)kReduceChunks * std::max({L1::NT, L2::NT, L3::NT});
}

hipError_t nn_forward(int n, int64_t nelem, const float *params, float *wt, const float *x0, float *a1, float *a2,
                      float *out, hipStream_t s)
{
    if (nelem <= 0) return hipSuccess;
    if (n == 3) return forward_t<3>(nelem, params, wt, x0, a1, a2, out, s);
    if (n == 4) return forward_t<4>(nelem, params, wt, x0, a1, a2, out, s);
    if (n == 5) return forward_t<5>(nelem, params, wt, x0, a1, a2, out, s);
    return hipErrorInvalidValue;
}

int64_t nn_pack16_bytes() { return (int64_t)kPackSteps * 64 * sizeof(h4_t); }

hipError_t nn_infer16(int n, int64_t nelem, const float *params, void *wpack, const double *r, const int32_t *emap,
                      const float *logk, const double *inv_mult, double scale, double *z, hipStream_t s)
{
    if (nelem <= 0) return hipSuccess;
    h4_t *wp = static_cast<h4_t *>(wpack);
    hipLaunchKernelGGL(k_pack16, dim3((kPackSteps * 64 + 255) / 256), dim3(256), 0, s, params, wp);
    // persistent workgroups (one element at a time each): enough to fill every CU several times over
    const unsigned nb = (unsigned)std::min<int64_t>(nelem, 256 * 8);
    if (n == 3) hipLaunchKernelGGL(k_net16<3>, dim3(nb), dim3(256), 0, s, nelem, r, emap, logk, wp, params, inv_mult, scale, z);
    else if (n == 4) hipLaunchKernelGGL(k_net16<4>, dim3(nb), dim3(256), 0, s, nelem, r, emap, logk, wp, params, inv_mult, scale, z);
    else if (n == 5) hipLaunchKernelGGL(k_net16<5>, dim3(nb), dim3(256), 0, s, nelem, r, emap, logk, wp, params, inv_mult, scale, z);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t nn_backward(int n, int64_t nelem, const float *params, const float *x0, const float *a1, const float *a2,
                       const float *gout, float *ga2, float *ga1, float *grads, float *wt, float *partial,
                       hipStream_t s)
{
    if (nelem <= 0) return hipSuccess;
    if (n == 3) return backward_t<3>(nelem, params, x0, a1, a2, gout, ga2, ga1, grads, wt, partial, s);
    if (n == 4) return backward_t<4>(nelem, params, x0, a1, a2, gout, ga2, ga1, grads, wt, partial, s);
    if (n == 5) return backward_t<5>(nelem, params, x0, a1, a2, gout, ga2, ga1, grads, wt, partial, s);
    return hipErrorInvalidValue;
}

hipError_t nn_input(int n, int64_t nelem, const double *r, const int32_t *emap, const float *logk, float *x0,
                    float *s, hipStream_t st)
{
    if (nelem <= 0) return hipSuccess;
    if (n == 3) hipLaunchKernelGGL(k_nn_input<3>, dim3(nelem), dim3(128), 0, st, nelem, r, emap, logk, x0, s);
    else if (n == 4) hipLaunchKernelGGL(k_nn_input<4>, dim3(nelem), dim3(128), 0, st, nelem, r, emap, logk, x0, s);
    else if (n == 5) hipLaunchKernelGGL(k_nn_input<5>, dim3(nelem), dim3(128), 0, st, nelem, r, emap, logk, x0, s);
    else return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t nn_output(int n, int64_t nelem, const float *out, const float *s, const int32_t *emap,
                     const double *inv_mult, double scale, double *z, hipStream_t st)
{
    const int P = n * n * n;
    const int64_t tot = nelem * P;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nn_output, dim3(nblk(tot)), dim3(256), 0, st, tot, P, out, s, emap, inv_mult, scale, z);
    return hipGetLastError();
}

hipError_t nn_output_grad(int n, int64_t nelem, const double *gz, const float *s, const int32_t *emap,
                          const double *inv_mult, float *gout, hipStream_t st)
{
    const int P = n * n * n;
    const int64_t tot = nelem * P;
    if (tot <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_nn_output_grad, dim3(nblk(tot)), dim3(256), 0, st, tot, P, gz, s, emap, inv_mult, gout);
    return hipGetLastError();
}

hipError_t nn_inv_mult(int n, int64_t nelem, int64_t ndof, const int32_t *emap, double *inv_mult, hipStream_t s)
{
    const int64_t tot = nelem * n * n * n;
    hipError_t e = vec_fill(inv_mult, 0.0, ndof, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_count, dim3(nblk(tot)), dim3(256), 0, s, tot, emap, inv_mult);
    hipLaunchKernelGGL(k_recip_or_zero, dim3(nblk(ndof)), dim3(256), 0, s, ndof, inv_mult);
    return hipGetLastError();
}

hipError_t nn_adam(float *p, float *g, float *m, float *v, int n, double lr, int step, hipStream_t s)
{
    const double bc1 = 1.0 - std::pow(0.9, step), bc2 = 1.0 - std::pow(0.999, step);
    hipLaunchKernelGGL(k_adam, dim3(nblk(n)), dim3(256), 0, s, p, g, m, v, n, (float)lr, (float)bc1, (float)bc2);
    return hipGetLastError();
}

hipError_t vec_fill_f32(float *y, float v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)std::min<int64_t>(nblk(n), 8192)), dim3(256), 0, s, y, v, n);
    return hipGetLastError();
}

hipError_t vec_sub(double *y, const double *a, const double *b, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_sub, dim3((unsigned)std::min<int64_t>(nblk(n), 8192)), dim3(256), 0, s, y, a, b, n);
    return hipGetLastError();
}
hipError_t vec_mul(double *y, const double *a, const double *b, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mul, dim3((unsigned)std::min<int64_t>(nblk(n), 8192)), dim3(256), 0, s, y, a, b, n);
    return hipGetLastError();
}

hipError_t vec_loss_scale(double *g, int64_t n, double *sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_loss_scale, dim3((unsigned)std::min<int64_t>(nblk(n), 8192)), dim3(256), 0, s, g, n, sc);
    return hipGetLastError();
}

hipError_t coarse_prolong(const BoxDims &b, const double *gll, const double *u1, double *uf, bool add, hipStream_t s)
{
    const int64_t nf = ((int64_t)b.nx * b.p + 1) * ((int64_t)b.ny * b.p + 1) * ((int64_t)b.nz * b.p + 1);
    hipLaunchKernelGGL(k_prolong, dim3(nblk(nf)), dim3(256), 0, s, b, gll, u1, uf, add ? 1 : 0);
    return hipGetLastError();
}

hipError_t coarse_restrict(const BoxDims &b, const double *gll, const double *rf, double *r1, double *t1, double *t2,
                           hipStream_t s)
{
    const int64_t Mx = (int64_t)b.nx * b.p + 1, My = (int64_t)b.ny * b.p + 1, Mz = (int64_t)b.nz * b.p + 1;
    const int64_t Cx = b.nx + 1, Cy = b.ny + 1, Cz = b.nz + 1;
    hipLaunchKernelGGL(k_restrict_axis, dim3(nblk(Cx * My * Mz)), dim3(256), 0, s, 0, b.nx, b.p, Mx, My, Mz, gll, rf, t1);
    hipLaunchKernelGGL(k_restrict_axis, dim3(nblk(Cx * Cy * Mz)), dim3(256), 0, s, 1, b.ny, b.p, Cx, My, Mz, gll, t1, t2);
    hipLaunchKernelGGL(k_restrict_axis, dim3(nblk(Cx * Cy * Cz)), dim3(256), 0, s, 2, b.nz, b.p, Cx, Cy, Mz, gll, t2, r1);
    return hipGetLastError();
}

hipError_t coarse_probe_vec(const BoxDims &b, int cls, double *v, hipStream_t s)
{
    const int64_t n1 = (int64_t)(b.nx + 1) * (b.ny + 1) * (b.nz + 1);
    hipLaunchKernelGGL(k_probe_vec, dim3(nblk(n1)), dim3(256), 0, s, b, cls, v);
    return hipGetLastError();
}

hipError_t coarse_probe_gather(const BoxDims &b, int cls, const double *y, const uint8_t *ess1, double *S,
                               hipStream_t s)
{
    const int64_t n1 = (int64_t)(b.nx + 1) * (b.ny + 1) * (b.nz + 1);
    hipLaunchKernelGGL(k_probe_gather, dim3(nblk(n1)), dim3(256), 0, s, b, cls, y, ess1, S);
    return hipGetLastError();
}

hipError_t coarse_dinv(int64_t n1, const double *S, double *dinv, hipStream_t s)
{
    hipLaunchKernelGGL(k_dinv_center, dim3(nblk(n1)), dim3(256), 0, s, n1, S, dinv);
    return hipGetLastError();
}

hipError_t coarse_pcg(const BoxDims &b, const double *S, const double *dinv, double *r1, double *u, double *z,
                      double *p0, double *p1, double *Ap, double *partial, CoarseScalars *sc, int iters,
                      hipStream_t s)
{
    const int64_t n1 = (int64_t)(b.nx + 1) * (b.ny + 1) * (b.nz + 1);
    const unsigned nb = (unsigned)((n1 + kCoarseThreads - 1) / kCoarseThreads);
    hipLaunchKernelGGL(k_cpcg_init, dim3(nb), dim3(kCoarseThreads), 0, s, n1, dinv, r1, u, z, p0, partial, sc);
    for (int k = 0; k < iters; ++k) {
        double *pin = (k & 1) ? p1 : p0, *pout = (k & 1) ? p0 : p1;
        hipLaunchKernelGGL(k_cpcg_a, dim3(nb), dim3(kCoarseThreads), 0, s, b, S, z, pin, pout, Ap, partial, sc);
        hipLaunchKernelGGL(k_cpcg_b, dim3(nb), dim3(kCoarseThreads), 0, s, n1, dinv, pout, Ap, u, r1, z, partial, sc);
    }
    return hipGetLastError();
}

}  // namespace hexpa
