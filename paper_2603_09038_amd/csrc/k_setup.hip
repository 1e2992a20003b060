// Setup kernels: quadrature-point data D (partial assembly, paper Sec. II-B), physical
// coordinates of quadrature points and nodes, and the load vector G^T B^T (w detJ f).
#include <hip/hip_runtime.h>

#include "geometry.h"
#include "internal.h"

namespace hexpa {

namespace {

// D at every (element, qp): diffusion w k adj(J) adj(J)^T / det J (rows of adj(J) are the
// cross products of the Jacobian columns), mass w k det J.  Layout [e][comp][qp].
// D at every (element, qp), layout [e][comp][qp]; flags a non-positive det J.
template <int OPS>
__global__ void k_setup_qdata_t(int64_t nelem, int q, const double *__restrict__ vert, const int32_t *__restrict__ hex,
                                const DevTables *__restrict__ tab, CoeffDev cf, double *__restrict__ qd,
                                int *__restrict__ bad)
{
    constexpr int NC = ((OPS & PA_DIFFUSION) ? 6 : 0) + ((OPS & PA_MASS) ? 1 : 0);
    const int q3 = q * q * q;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nelem * q3) return;
    const int64_t e = idx / q3;
    const int r = (int)(idx - e * q3);
    const int a = r % q, b = (r / q) % q, c = r / (q * q);
    Hex h;
    load_hex(vert, hex, e, h);
    double dv[NC];
    const double det = qp_data<OPS>(h, tab->x[a], tab->x[b], tab->x[c], tab->w[a] * tab->w[b] * tab->w[c], cf, dv);
    if (!(det > 0.0)) *bad = 1;
    double *out = qd + e * (int64_t)NC * q3 + r;
#pragma unroll
    for (int m = 0; m < NC; ++m) out[m * q3] = dv[m];
}

__global__ void k_qpoints(int64_t nelem, int q, const double *__restrict__ vert, const int32_t *__restrict__ hex,
                          const DevTables *__restrict__ tab, double *__restrict__ out)
{
    const int q3 = q * q * q;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nelem * q3) return;
    const int64_t e = idx / q3;
    const int r = (int)(idx - e * q3);
    Hex h;
    load_hex(vert, hex, e, h);
    double x[3], J[3][3];
    map_point(h, tab->x[r % q], tab->x[(r / q) % q], tab->x[r / (q * q)], x, J);
    out[idx * 3 + 0] = x[0];
    out[idx * 3 + 1] = x[1];
    out[idx * 3 + 2] = x[2];
}

__global__ void k_nodes(int64_t nelem, int d, const double *__restrict__ vert, const int32_t *__restrict__ hex,
                        const int32_t *__restrict__ emap, const DevTables *__restrict__ tab, double *__restrict__ out)
{
    const int d3 = d * d * d;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nelem * d3) return;
    const int64_t e = idx / d3;
    const int I = (int)(idx - e * d3);
    Hex h;
    load_hex(vert, hex, e, h);
    double x[3], J[3][3];
    map_point(h, tab->nodes[I % d], tab->nodes[(I / d) % d], tab->nodes[I / (d * d)], x, J);
    const int64_t g = emap[idx];
    out[g * 3 + 0] = x[0];
    out[g * 3 + 1] = x[1];
    out[g * 3 + 2] = x[2];
}

// w detJ f at every quadrature point (in place into tmp).
__global__ void k_load_qp(int64_t nelem, int q, const double *__restrict__ vert, const int32_t *__restrict__ hex,
                          const DevTables *__restrict__ tab, const double *__restrict__ f, double *__restrict__ tmp)
{
    const int q3 = q * q * q;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nelem * q3) return;
    const int64_t e = idx / q3;
    const int r = (int)(idx - e * q3);
    const int a = r % q, b = (r / q) % q, c = r / (q * q);
    Hex h;
    load_hex(vert, hex, e, h);
    double x[3], J[3][3];
    map_point(h, tab->x[a], tab->x[b], tab->x[c], x, J);
    const double det = J[0][0] * (J[1][1] * J[2][2] - J[2][1] * J[1][2]) - J[1][0] * (J[0][1] * J[2][2] - J[2][1] * J[0][2]) +
                       J[2][0] * (J[0][1] * J[1][2] - J[1][1] * J[0][2]);
    tmp[idx] = tab->w[a] * tab->w[b] * tab->w[c] * det * f[idx];
}

// b += G^T B^T tmp, one thread per (element, local node), contraction over all qps.
__global__ void k_load_scatter(int64_t nelem, int d, int q, const int32_t *__restrict__ emap,
                               const DevTables *__restrict__ tab, const double *__restrict__ tmp,
                               double *__restrict__ bvec)
{
    const int d3 = d * d * d, q3 = q * q * q;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nelem * d3) return;
    const int64_t e = idx / d3;
    const int I = (int)(idx - e * d3);
    const int i = I % d, j = (I / d) % d, k = I / (d * d);
    const double *t = tmp + e * q3;
    double acc = 0.0;
    for (int c = 0; c < q; ++c)
        for (int b = 0; b < q; ++b) {
            const double bc = tab->B[b * d + j] * tab->B[c * d + k];
            for (int a = 0; a < q; ++a) acc += tab->B[a * d + i] * bc * t[a + q * (b + q * c)];
        }
    unsafeAtomicAdd(bvec + emap[idx], acc);
}

// log kappa at every (element, local node), the network's second input channel.
__global__ void k_logk_tiles(int64_t nelem, int d, const double *__restrict__ vert, const int32_t *__restrict__ hex,
                             const DevTables *__restrict__ tab, CoeffDev cf, float *__restrict__ out)
{
    const int d3 = d * d * d;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= nelem * d3) return;
    const int64_t e = idx / d3;
    const int I = (int)(idx - e * d3);
    Hex h;
    load_hex(vert, hex, e, h);
    double x[3], J[3][3];
    map_point(h, tab->nodes[I % d], tab->nodes[(I / d) % d], tab->nodes[I / (d * d)], x, J);
    out[idx] = (float)log(coeff_eval(cf, x));
}

inline unsigned nblk(int64_t n) { return (unsigned)((n + 255) / 256); }

}  // namespace

hipError_t logk_tiles(const pa_op *op, float *out, hipStream_t s)
{
    const int64_t n = (int64_t)op->nelem * op->d * op->d * op->d;
    hipLaunchKernelGGL(k_logk_tiles, dim3(nblk(n)), dim3(256), 0, s, (int64_t)op->nelem, op->d, op->d_vert,
                       op->d_hex, op->d_tab, op->coeff, out);
    return hipGetLastError();
}

hipError_t launch_setup_qdata(const pa_op *op, const CoeffDev &cf, int *d_bad, hipStream_t s)
{
    const int64_t n = (int64_t)op->nelem * op->q * op->q * op->q;
    switch (op->ops) {
    case PA_MASS:
        hipLaunchKernelGGL(k_setup_qdata_t<PA_MASS>, dim3(nblk(n)), dim3(256), 0, s, (int64_t)op->nelem, op->q,
                           op->d_vert, op->d_hex, op->d_tab, cf, op->d_qdata, d_bad);
        break;
    case PA_DIFFUSION:
        hipLaunchKernelGGL(k_setup_qdata_t<PA_DIFFUSION>, dim3(nblk(n)), dim3(256), 0, s, (int64_t)op->nelem, op->q,
                           op->d_vert, op->d_hex, op->d_tab, cf, op->d_qdata, d_bad);
        break;
    default:
        hipLaunchKernelGGL(k_setup_qdata_t<PA_MASS | PA_DIFFUSION>, dim3(nblk(n)), dim3(256), 0, s, (int64_t)op->nelem,
                           op->q, op->d_vert, op->d_hex, op->d_tab, cf, op->d_qdata, d_bad);
    }
    return hipGetLastError();
}

hipError_t launch_qpoints(const pa_op *op, double *xyz, hipStream_t s)
{
    const int64_t n = (int64_t)op->nelem * op->q * op->q * op->q;
    hipLaunchKernelGGL(k_qpoints, dim3(nblk(n)), dim3(256), 0, s, (int64_t)op->nelem, op->q, op->d_vert, op->d_hex,
                       op->d_tab, xyz);
    return hipGetLastError();
}

hipError_t launch_nodes(const pa_op *op, double *xyz, hipStream_t s)
{
    const int64_t n = (int64_t)op->nelem * op->d * op->d * op->d;
    hipLaunchKernelGGL(k_nodes, dim3(nblk(n)), dim3(256), 0, s, (int64_t)op->nelem, op->d, op->d_vert, op->d_hex,
                       op->d_elem_dofs, op->d_tab, xyz);
    return hipGetLastError();
}

hipError_t launch_load(const pa_op *op, const double *fq, double *b, hipStream_t s)
{
    const int64_t nq = (int64_t)op->nelem * op->q * op->q * op->q;
    const int64_t nd = (int64_t)op->nelem * op->d * op->d * op->d;
    double *tmp = nullptr;
    hipError_t err = hipMallocAsync((void **)&tmp, nq * sizeof(double), s);
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_load_qp, dim3(nblk(nq)), dim3(256), 0, s, (int64_t)op->nelem, op->q, op->d_vert, op->d_hex,
                       op->d_tab, fq, tmp);
    if ((err = vec_fill(b, 0.0, op->ndof, s)) != hipSuccess) return err;
    hipLaunchKernelGGL(k_load_scatter, dim3(nblk(nd)), dim3(256), 0, s, (int64_t)op->nelem, op->d, op->q,
                       op->d_elem_dofs, op->d_tab, tmp, b);
    err = hipGetLastError();
    hipError_t e2 = hipFreeAsync(tmp, s);
    return err != hipSuccess ? err : e2;
}

}  // namespace hexpa
