// Vector kernels and the fused FP64 CG update kernels (deterministic two-stage reductions).
#include <hip/hip_runtime.h>

#include "k_vec.h"

namespace hexpa {

namespace {

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

__global__ void k_fill(double *y, double v, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = v;
}
__global__ void k_copy(double *y, const double *x, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) y[i] = x[i];
}
__global__ void k_set_list(double *y, double v, const int32_t *list, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[list[i]] = v;
}
__global__ void k_copy_list(double *y, const double *x, const int32_t *list, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[list[i]] = x[list[i]];
}

// Block-wide sum of NV values per thread in a fixed tree order (bitwise reproducible).
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

// partial[b] = sum over this block's strided range of x.y
__global__ void k_dot_partial(const double *__restrict__ x, const double *__restrict__ y, int64_t n, double *partial)
{
    __shared__ double sh[256];
    double v[1] = {0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        v[0] = fma(x[i], y[i], v[0]);
    block_sum<1>(v, sh);
    if (threadIdx.x == 0) partial[blockIdx.x] = v[0];
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

// x += alpha p; r -= alpha Ap; partial sums of (r . dinv r) and (r . r).
__global__ void k_cg_update1(double *__restrict__ x, double *__restrict__ r, const double *__restrict__ p,
                             const double *__restrict__ Ap, const double *__restrict__ dinv, int64_t n,
                             const CgScalars *__restrict__ s, double *partial)
{
    __shared__ double sh[2 * 256];
    const double alpha = s->alpha;
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = fma(alpha, p[i], x[i]);
        const double ri = fma(-alpha, Ap[i], r[i]);
        r[i] = ri;
        const double zi = dinv ? dinv[i] * ri : ri;
        v[0] = fma(ri, zi, v[0]);
        v[1] = fma(ri, ri, v[1]);
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = v[0];
        partial[2 * blockIdx.x + 1] = v[1];
    }
}

// beta = rz_new / rz; rz = rz_new; record ||r||^2 for iteration `it`.
__global__ void k_cg_beta(const double *partial, int nb, CgScalars *s, double *rr_hist, int it)
{
    __shared__ double sh[2 * 256];
    double v[2] = {0.0, 0.0};
    for (int i = threadIdx.x; i < nb; i += 256) {
        v[0] += partial[2 * i];
        v[1] += partial[2 * i + 1];
    }
    block_sum<2>(v, sh);
    if (threadIdx.x == 0) {
        const double rz_new = v[0];
        if (!isfinite(rz_new) || !isfinite(v[1])) s->breakdown = 1;
        s->beta = (s->rz != 0.0) ? rz_new / s->rz : 0.0;
        s->rz = rz_new;
        s->rr = v[1];
        rr_hist[2 * it] = v[1];
        rr_hist[2 * it + 1] = (double)s->breakdown;
    }
}

// p = dinv r + beta p
__global__ void k_cg_update2(double *__restrict__ p, const double *__restrict__ r, const double *__restrict__ dinv,
                             int64_t n, const CgScalars *__restrict__ s)
{
    const double beta = s->beta;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double zi = dinv ? dinv[i] * r[i] : r[i];
        p[i] = fma(beta, p[i], zi);
    }
}

// r = b - Ax (in place into Ax), and partial sums of r . dinv r and r . r; p = dinv r.
__global__ void k_cg_init(const double *__restrict__ b, double *__restrict__ r, double *__restrict__ p,
                          const double *__restrict__ dinv, int64_t n, double *partial)
{
    __shared__ double sh[2 * 256];
    double v[2] = {0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ri = b[i] - r[i];
        r[i] = ri;
        const double zi = dinv ? dinv[i] * ri : ri;
        p[i] = zi;
        v[0] = fma(ri, zi, v[0]);
        v[1] = fma(ri, ri, v[1]);
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

}  // namespace

hipError_t vec_fill(double *y, double v, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(min(nblk(n), 8192u)), dim3(256), 0, s, y, v, n);
    return hipGetLastError();
}
hipError_t vec_copy(double *y, const double *x, int64_t n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy, dim3(min(nblk(n), 8192u)), dim3(256), 0, s, y, x, n);
    return hipGetLastError();
}
hipError_t vec_set_list(double *y, double v, const int32_t *list, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_set_list, dim3(nblk(n)), dim3(256), 0, s, y, v, list, n);
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
hipError_t vec_dot(const double *x, const double *y, int64_t n, double *partial, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(256), 0, s, x, y, n, partial);
    hipLaunchKernelGGL(k_reduce_to, dim3(1), dim3(256), 0, s, partial, kRedBlocks, 1, out);
    return hipGetLastError();
}

hipError_t cg_init(const double *b, double *r, double *p, const double *dinv, int64_t n, double *partial,
                   CgScalars *sc, double *hist, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_init, dim3(kRedBlocks), dim3(256), 0, s, b, r, p, dinv, n, partial);
    hipLaunchKernelGGL(k_cg_init_scalars, dim3(1), dim3(256), 0, s, partial, kRedBlocks, sc, hist);
    return hipGetLastError();
}
hipError_t cg_alpha(const double *p, const double *Ap, int64_t n, double *partial, CgScalars *sc, hipStream_t s)
{
    hipLaunchKernelGGL(k_dot_partial, dim3(kRedBlocks), dim3(256), 0, s, p, Ap, n, partial);
    hipLaunchKernelGGL(k_cg_alpha, dim3(1), dim3(256), 0, s, partial, kRedBlocks, sc);
    return hipGetLastError();
}
hipError_t cg_update(double *x, double *r, double *p, const double *Ap, const double *dinv, int64_t n,
                     double *partial, CgScalars *sc, double *hist, int it, hipStream_t s)
{
    hipLaunchKernelGGL(k_cg_update1, dim3(kRedBlocks), dim3(256), 0, s, x, r, p, Ap, dinv, n, sc, partial);
    hipLaunchKernelGGL(k_cg_beta, dim3(1), dim3(256), 0, s, partial, kRedBlocks, sc, hist, it);
    hipLaunchKernelGGL(k_cg_update2, dim3(kRedBlocks), dim3(256), 0, s, p, r, dinv, n, sc);
    return hipGetLastError();
}

}  // namespace hexpa
