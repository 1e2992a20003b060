// Vector kernels and the fused CG update kernels.  Vectors are FP64 or FP32 (the
// mixed-precision inner solve); every reduction accumulates in FP64 with a fixed block
// count and a fixed tree order, so sums are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "k_vec.h"

namespace hexpa {

// Grid-stride loops of the CG vector kernels keep kUnroll strides of loads in flight per
// thread (the order of every per-thread sum is unchanged).
constexpr int kUnroll = 4;

namespace {

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

template <class T>
__global__ void k_fill(T *y, T v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = v;
}
__global__ void k_copy(double *y, const double *x, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = x[i];
}
template <class T>
__global__ void k_set_list(T *y, T v, const int32_t *list, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[list[i]] = v;
}
__global__ void k_copy_list(double *y, const double *x, const int32_t *list, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[list[i]] = x[list[i]];
}

// Block-wide sum of NV values per thread in a fixed tree order.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double *sh /*[NV][256]*/)
{
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NV; ++k) sh[k * 256 + t] = v[k];
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (t < s)
#pragma unroll
            for (int k = 0; k < NV; ++k) sh[k * 256 + t] += sh[k * 256 + t + s];
        __syncthreads();
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) v[k] = sh[k * 256];
}

template <class T>
__global__ void k_dot_partial(const T *__restrict__ x, const T *__restrict__ y, int64_t n, double *partial)
{
    __shared__ double sh[256];
    double v[1] = {0.0};
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kUnroll - 1) * st < n; i += kUnroll * st) {  // loads of kUnroll strides in flight
        T xv[kUnroll], yv[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            xv[u] = x[i + u * st];
            yv[u] = y[i + u * st];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) v[0] = fma((double)xv[u], (double)yv[u], v[0]);
    }
    for (; i < n; i += st) v[0] = fma((double)x[i], (double)y[i], v[0]);
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

__global__ void k_maxabs_partial(const double *__restrict__ x, int64_t n, double *partial)
{
    __shared__ double sh[256];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        m = fmax(m, fabs(x[i]));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = sh[0];
}

__global__ void k_max_to(const double *partial, int nb, double *out)
{
    __shared__ double sh[256];
    double m = 0.0;
    for (int i = threadIdx.x; i < nb; i += 256) m = fmax(m, partial[i]);
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = sh[0];
}

__global__ void k_reduce_to(const double *partial, int nb, int stride, double *out)
{
    __shared__ double sh[256];
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nb; i += 256) v[0] += partial[i * stride];
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) *out = v[0];
}

// alpha = rz / pAp from the partial sums of p.Ap; flags breakdown.
__global__ void k_cg_alpha(const double *partial, int nb, CgScalars *s)
{
    __shared__ double sh[256];
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nb; i += 256) v[0] += partial[i];
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) {
        const double pAp = v[0];
        s->pAp = pAp;
        if (!(pAp > 0.0) || !isfinite(pAp) || !isfinite(s->rz)) {
            s->breakdown = 1;
            s->alpha = 0.0;
        } else {
            s->alpha = s->rz / pAp;
        }
    }
}

// alpha = rz / (p . Ap) from the partial sums of p . Ap, formed identically (same order) in
// every block; x += alpha p; r -= alpha Ap; rz_prev = rz; partial sums of (r . dinv r) and
// (r . r) into rz_part.
template <class T>
__global__ void k_cg_update1(T *__restrict__ x, T *__restrict__ r, const T *__restrict__ p, const T *__restrict__ Ap,
                             const T *__restrict__ dinv, int64_t n, CgScalars *__restrict__ s,
                             const double *__restrict__ pap_part, int nb, double *__restrict__ rz_part)
{
    __shared__ double sh[2 * 256];
    double a[1] = {0.0};
    for (int i = threadIdx.x; i < nb; i += 256) a[0] += pap_part[i];
    block_sum<1>(a, sh);
    const double pAp = a[0], rz = s->rz;
    const bool bad = !(pAp > 0.0) || !isfinite(pAp) || !isfinite(rz);
    const double alpha = bad ? 0.0 : rz / pAp;
    // After a breakdown (this step's, seen identically by every block, or an earlier one:
    // the flag is sticky) x and r keep their last values, so the caller gets the last
    // finite iterate even when p or Ap hold non-finite entries (0 * NaN is NaN).
    const bool frozen = bad || s->breakdown != 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        s->pAp = pAp;
        s->alpha = alpha;
        s->rz_prev = rz;
        if (bad) s->breakdown = 1;
    }
    __syncthreads();  // sh is reused below
    double v[2] = {0.0, 0.0};
    auto one = [&](int64_t i, T pi, T xi, T ai, T r0, T di) {
        T ri = r0;
        if (!frozen) {
            x[i] = (T)fma(alpha, (double)pi, (double)xi);
            ri = (T)fma(-alpha, (double)ai, (double)r0);
            r[i] = ri;
        }
        const double zi = dinv ? (double)(di * ri) : (double)ri;
        v[0] = fma((double)ri, zi, v[0]);
        v[1] = fma((double)ri, (double)ri, v[1]);
    };
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kUnroll - 1) * st < n; i += kUnroll * st) {  // same order, loads batched
        T pv[kUnroll], xv[kUnroll], av[kUnroll], rv[kUnroll], dv[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t j = i + u * st;
            pv[u] = p[j];
            xv[u] = x[j];
            av[u] = Ap[j];
            rv[u] = r[j];
            dv[u] = dinv ? dinv[j] : T(1);
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) one(i + u * st, pv[u], xv[u], av[u], rv[u], dv[u]);
    }
    for (; i < n; i += st) one(i, p[i], x[i], Ap[i], r[i], dinv ? dinv[i] : T(1));
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        rz_part[2 * blockIdx.x] = v[0];
        rz_part[2 * blockIdx.x + 1] = v[1];
    }
}

// beta = rz_new / (rz_prev f) from the partial sums of (r . dinv r, r . r), formed in every
// block; p = dinv r + beta p; Ap = 0 for the next apply (if given).  Block 0 stores
// rz = rz_new, rr, beta and hist[2 it] = r.r, hist[2 it + 1] = breakdown flag.  f != 1 when
// r and p were rescaled by f since rz_prev was taken (rz scales by f^2, the old direction
// by f: one f folded into beta rescales p inside the update).
template <class T>
__global__ void k_cg_update2(T *__restrict__ p, const T *__restrict__ r, const T *__restrict__ dinv,
                             T *__restrict__ Ap_zero, int64_t n, CgScalars *__restrict__ s,
                             const double *__restrict__ rz_part, int nb, double *__restrict__ rr_hist, int it, double f)
{
    __shared__ double sh[2 * 256];
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += 256) {
        v[0] += rz_part[2 * i];
        v[1] += rz_part[2 * i + 1];
    }
    block_sum<2>(v, sh);
    const double rz_new = v[0], rzp = s->rz_prev;
    const double beta = (rzp != 0.0) ? rz_new / (rzp * f) : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (!isfinite(rz_new) || !isfinite(v[1])) s->breakdown = 1;
        s->beta = beta;
        s->rz = rz_new;
        s->rr = v[1];
        rr_hist[2 * it] = v[1];
        rr_hist[2 * it + 1] = (double)s->breakdown;
    }
    const int64_t st = (int64_t)gridDim.x * blockDim.x;
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (; i + (kUnroll - 1) * st < n; i += kUnroll * st) {  // loads batched
        T rv[kUnroll], dv[kUnroll], pv[kUnroll];
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t j = i + u * st;
            rv[u] = r[j];
            dv[u] = dinv ? dinv[j] : T(1);
            pv[u] = p[j];
        }
#pragma unroll
        for (int u = 0; u < kUnroll; ++u) {
            const int64_t j = i + u * st;
            const double zi = dinv ? (double)(dv[u] * rv[u]) : (double)rv[u];
            p[j] = (T)fma(beta, (double)pv[u], zi);
            if (Ap_zero) Ap_zero[j] = T(0);
        }
    }
    for (; i < n; i += st) {
        const double zi = dinv ? (double)(dinv[i] * r[i]) : (double)r[i];
        p[i] = (T)fma(beta, (double)p[i], zi);
        if (Ap_zero) Ap_zero[i] = T(0);
    }
}

// r = b - r_in (r holds A x on entry; b == nullptr: r unchanged) and partial sums of
// r . dinv r and r . r; p = dinv r (p == nullptr: not written).
template <class T>
__global__ void k_cg_init(const T *__restrict__ b, T *__restrict__ r, T *__restrict__ p, const T *__restrict__ dinv,
                          int64_t n, double *partial)
{
    __shared__ double sh[2 * 256];
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const T ri = b ? (T)(b[i] - r[i]) : r[i];
        r[i] = ri;
        const T zi = dinv ? dinv[i] * ri : ri;
        if (p) p[i] = zi;
        v[0] = fma((double)ri, (double)zi, v[0]);
        v[1] = fma((double)ri, (double)ri, v[1]);
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = v[0];
        partial[2 * blockIdx.x + 1] = v[1];
    }
}

__global__ void k_cg_init_scalars(const double *partial, int nb, CgScalars *s, double *rr_hist)
{
    __shared__ double sh[2 * 256];
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += 256) {
        v[0] += partial[2 * i];
        v[1] += partial[2 * i + 1];
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        s->rz = v[0];
        s->rr = v[1];
        s->breakdown = 0;
        s->alpha = s->beta = s->pAp = 0.0;
        rr_hist[0] = v[1];
        rr_hist[1] = 0.0;
    }
}

__global__ void k_recip(double *y, const double *x, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = 1.0 / x[i];
}
__global__ void k_to_f32(float *y, const double *x, double scale, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)(x[i] * scale);
}
__global__ void k_axpy_f32(double *x, double a, const float *d, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        x[i] = fma(a, (double)d[i], x[i]);
}

// ---- flexible CG (FCG(1)) pieces
// x += alpha p; rold = r; r -= alpha Ap; partial sums of r.r.  Once a breakdown has been
// flagged (sticky; no block of this kernel writes the flag) x, r and rold are left as they
// are: a non-finite preconditioner output reaches p before the host sees the flag, and
// alpha = 0 would still turn x into 0 * NaN.  The fallback restarts from that x.
__global__ void k_fcg_update(double *__restrict__ x, double *__restrict__ r, double *__restrict__ rold,
                             const double *__restrict__ p, const double *__restrict__ Ap, int64_t n,
                             const CgScalars *__restrict__ s, double *partial)
{
    __shared__ double sh[256];
    const double alpha = s->alpha;
    const bool frozen = s->breakdown != 0;
    double v[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = r[i];
        double rn = ri;
        if (!frozen) {
            x[i] = fma(alpha, p[i], x[i]);
            rold[i] = ri;
            rn = fma(-alpha, Ap[i], ri);
            r[i] = rn;
        }
        v[0] = fma(rn, rn, v[0]);
    }
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
}

__global__ void k_fcg_rr(const double *partial, int nb, CgScalars *s, double *rr_hist, int it)
{
    __shared__ double sh[256];
    double v[1] = {0.0};
    for (int i = threadIdx.x; i < nb; i += 256) v[0] += partial[i];
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) {
        if (!isfinite(v[0])) s->breakdown = 1;
        s->rr = v[0];
        rr_hist[2 * it] = v[0];
        rr_hist[2 * it + 1] = (double)s->breakdown;
    }
}

// partial sums of z.r and z.rold (rold may be null)
__global__ void k_fcg_dots(const double *__restrict__ z, const double *__restrict__ r, const double *__restrict__ rold,
                           int64_t n, double *partial)
{
    __shared__ double sh[2 * 256];
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        v[0] = fma(z[i], r[i], v[0]);
        if (rold) v[1] = fma(z[i], rold[i], v[1]);
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = v[0];
        partial[2 * blockIdx.x + 1] = v[1];
    }
}

// beta = (z.r - z.rold) / rz (0 for the first direction); rz = z.r
__global__ void k_fcg_beta(const double *partial, int nb, int first, CgScalars *s)
{
    __shared__ double sh[2 * 256];
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += 256) {
        v[0] += partial[2 * i];
        v[1] += partial[2 * i + 1];
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        const double zr = v[0], zro = v[1];
        if (!isfinite(zr) || !isfinite(zro)) s->breakdown = 1;
        s->beta = (first || s->rz == 0.0) ? 0.0 : (zr - zro) / s->rz;
        s->rz = zr;
    }
}

// p = z + beta p (p = z for the first direction)
__global__ void k_fcg_p(double *__restrict__ p, const double *__restrict__ z, int64_t n, int first,
                        const CgScalars *__restrict__ s)
{
    const double beta = s->beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = first ? z[i] : fma(beta, p[i], z[i]);
}

}  // namespace

template <class T>
hipError_t vec_fill_t(T *y, T v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<T>, dim3(min(nblk(n), 8192u)), dim3(256), 0, s, y, v, n);
    return hipGetLastError();
}
hipError_t vec_fill(double *y, double v, int64_t n, hipStream_t s) { return vec_fill_t<double>(y, v, n, s); }
hipError_t vec_fill(float *y, float v, int64_t n, hipStream_t s) { return vec_fill_t<float>(y, v, n, s); }
hipError_t vec_copy(double *y, const double *x, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(min(nblk(n), 8192u)), dim3(256), 0, s, y, x, n);
    return hipGetLastError();
}
hipError_t vec_set_list(double *y, double v, const int32_t *list, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_list<double>, dim3(nblk(n)), dim3(256), 0, s, y, v, list, n);
    return hipGetLastError();
}
hipError_t vec_set_list(float *y, float v, const int32_t *list, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_list<float>, dim3(nblk(n)), dim3(256), 0, s, y, v, list, n);
    return hipGetLastError();
}
hipError_t vec_zero_list(double *y, const int32_t *list, int n, hipStream_t s) { return vec_set_list(y, 0.0, list, n, s); }
hipError_t vec_copy_list(double *y, const double *x, const int32_t *list, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_list, dim3(nblk(n)), dim3(256), 0, s, y, x, list, n);
    return hipGetLastError();
}
hipError_t vec_recip(double *y, const double *x, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_recip, dim3(min(nblk(n), 8192u)), dim3(256), 0, s, y, x, n);
    return hipGetLastError();
}
hipError_t vec_to_f32(float *y, const double *x, double scale, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_to_f32, dim3(min(nblk(n), 8192u)), dim3(256), 0, s, y, x, scale, n);
    return hipGetLastError();
}
hipError_t vec_axpy_f32(double *x, double a, const float *d, int64_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_axpy_f32, dim3(min(nblk(n), 8192u)), dim3(256), 0, s, x, a, d, n);
    return hipGetLastError();
}
template <class T>
hipError_t vec_dot(const T *x, const T *y, int64_t n, double *partial, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(256), 0, s, x, y, n, partial);
    hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(256), 0, s, partial, kRedBlocks, 1, out);
    return hipGetLastError();
}
template hipError_t vec_dot<double>(const double *, const double *, int64_t, double *, double *, hipStream_t);
template hipError_t vec_dot<float>(const float *, const float *, int64_t, double *, double *, hipStream_t);

hipError_t vec_maxabs(const double *x, int64_t n, double *partial, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_maxabs_partial, dim3(kRedBlocks), dim3(256), 0, s, x, n, partial);
    hipLaunchKernelGGL(k_max_to, dim3(1), dim3(256), 0, s, partial, kRedBlocks, out);
    return hipGetLastError();
}

template <class T>
hipError_t cg_init(const T *b, T *r, T *p, const T *dinv, int64_t n, double *partial, CgScalars *sc, double *hist,
                   hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_init<T>, dim3(kRedBlocks), dim3(256), 0, s, b, r, p, dinv, n, partial);
    hipLaunchKernelGGL(k_cg_init_scalars, dim3(1), dim3(256), 0, s, partial, kRedBlocks, sc, hist);
    return hipGetLastError();
}
template <class T>
hipError_t cg_alpha(const T *p, const T *Ap, int64_t n, double *partial, CgScalars *sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(256), 0, s, p, Ap, n, partial);
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, s, partial, kRedBlocks, sc);
    return hipGetLastError();
}
template <class T>
hipError_t cg_pap(const T *p, const T *Ap, int64_t n, double *pap_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial<T>, dim3(kRedBlocks), dim3(256), 0, s, p, Ap, n, pap_part);
    return hipGetLastError();
}
template <class T>
hipError_t cg_update_xr(T *x, T *r, const T *p, const T *Ap, const T *dinv, int64_t n, const double *pap_part,
                        double *rz_part, CgScalars *sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_update1<T>, dim3(kRedBlocks), dim3(256), 0, s, x, r, p, Ap, dinv, n, sc, pap_part,
                       kRedBlocks, rz_part);
    return hipGetLastError();
}
template <class T>
hipError_t cg_rz_partials(const T *r, const T *dinv, int64_t n, double *rz_part, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_init<T>, dim3(kRedBlocks), dim3(256), 0, s, nullptr, const_cast<T *>(r), nullptr, dinv, n,
                       rz_part);
    return hipGetLastError();
}
template <class T>
hipError_t cg_update_dir(T *p, const T *r, const T *dinv, T *Ap_zero, int64_t n, const double *rz_part, CgScalars *sc,
                         double *hist, int it, double f, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_update2<T>, dim3(kRedBlocks), dim3(256), 0, s, p, r, dinv, Ap_zero, n, sc, rz_part,
                       kRedBlocks, hist, it, f);
    return hipGetLastError();
}
#define HEXPA_INST(T)                                                                                           \
    template hipError_t cg_init<T>(const T *, T *, T *, const T *, int64_t, double *, CgScalars *, double *,   \
                                   hipStream_t);                                                               \
    template hipError_t cg_alpha<T>(const T *, const T *, int64_t, double *, CgScalars *, hipStream_t);         \
    template hipError_t cg_pap<T>(const T *, const T *, int64_t, double *, hipStream_t);                      \
    template hipError_t cg_update_xr<T>(T *, T *, const T *, const T *, const T *, int64_t, const double *,    \
                                        double *, CgScalars *, hipStream_t);                                   \
    template hipError_t cg_rz_partials<T>(const T *, const T *, int64_t, double *, hipStream_t);              \
    template hipError_t cg_update_dir<T>(T *, const T *, const T *, T *, int64_t, const double *, CgScalars *, \
                                         double *, int, double, hipStream_t);
HEXPA_INST(double)
HEXPA_INST(float)

hipError_t fcg_update(double *x, double *r, double *rold, const double *p, const double *Ap, int64_t n,
                      double *partial, CgScalars *sc, double *hist, int it, hipStream_t s)
{
    hipLaunchKernelGGL(k_fcg_update, dim3(kRedBlocks), dim3(256), 0, s, x, r, rold, p, Ap, n, sc, partial);
    hipLaunchKernelGGL(k_fcg_rr, dim3(1), dim3(256), 0, s, partial, kRedBlocks, sc, hist, it);
    return hipGetLastError();
}

hipError_t fcg_direction(const double *z, const double *r, const double *rold, double *p, int64_t n, double *partial,
                         CgScalars *sc, hipStream_t s)
{
    const int first = rold ? 0 : 1;
    hipLaunchKernelGGL(k_fcg_dots, dim3(kRedBlocks), dim3(256), 0, s, z, r, rold, n, partial);
    hipLaunchKernelGGL(k_fcg_beta, dim3(1), dim3(256), 0, s, partial, kRedBlocks, first, sc);
    hipLaunchKernelGGL(k_fcg_p, dim3(kRedBlocks), dim3(256), 0, s, p, z, n, first, sc);
    return hipGetLastError();
}

}  // namespace hexpa
