// Setup kernels: quadrature-point data D (partial assembly, paper Sec. II-B), physical
// coordinates of quadrature points and nodes, and the load vector G^T B^T (w detJ f).
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hexpa {

namespace {

// Trilinear geometry of one hexahedron: corner c = a + 2b + 4c' at reference vertex (a,b,c').
struct Hex {
    double X[8][3];
};

__device__ inline void load_hex(const double *__restrict__ vert, const int32_t *__restrict__ hex, int64_t e, Hex &h)
{
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int64_t v = hex[e * 8 + c];
#pragma unroll
        for (int r = 0; r < 3; ++r) h.X[c][r] = vert[v * 3 + r];
    }
}

// Position and Jacobian columns: dx/dxi_s is the blend of the four edge vectors along s.
__device__ inline void map_point(const Hex &h, double u, double v, double w, double x[3], double J[3][3])
{
    const double um = 1.0 - u, vm = 1.0 - v, wm = 1.0 - w;
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        auto P = [&](int c) { return h.X[c][r]; };
        // edges along xi_1 (corners differing in bit 0), weighted by the other two coordinates
        J[r][0] = vm * wm * (P(1) - P(0)) + v * wm * (P(3) - P(2)) + vm * w * (P(5) - P(4)) + v * w * (P(7) - P(6));
        J[r][1] = um * wm * (P(2) - P(0)) + u * wm * (P(3) - P(1)) + um * w * (P(6) - P(4)) + u * w * (P(7) - P(5));
        J[r][2] = um * vm * (P(4) - P(0)) + u * vm * (P(5) - P(1)) + um * v * (P(6) - P(2)) + u * v * (P(7) - P(3));
        x[r] = wm * (vm * (um * P(0) + u * P(1)) + v * (um * P(2) + u * P(3))) +
               w * (vm * (um * P(4) + u * P(5)) + v * (um * P(6) + u * P(7)));
    }
}

__device__ inline double coeff_eval(const CoeffDev &cf, const double x[3])
{
    if (cf.kind == PA_COEFF_CONST) return cf.value;
    if (cf.kind == PA_COEFF_SINE) {
        const double k = cf.freq * M_PI;
        return cf.value + cf.amp * sin(k * x[0]) * sin(k * x[1]) * sin(k * x[2]);
    }
    // grid: trilinear interpolation, clamped to [0,1]^3
    const int n[3] = {cf.gx, cf.gy, cf.gz};
    int i0[3];
    double f[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        double t = fmin(fmax(x[s], 0.0), 1.0) * (n[s] - 1);
        int i = (int)t;
        i = min(i, n[s] - 2);
        i0[s] = i;
        f[s] = t - i;
    }
    auto at = [&](int dx, int dy, int dz) {
        return cf.grid[(int64_t)(i0[0] + dx) + (int64_t)n[0] * ((i0[1] + dy) + (int64_t)n[1] * (i0[2] + dz))];
    };
    const double c00 = at(0, 0, 0) + f[0] * (at(1, 0, 0) - at(0, 0, 0));
    const double c10 = at(0, 1, 0) + f[0] * (at(1, 1, 0) - at(0, 1, 0));
    const double c01 = at(0, 0, 1) + f[0] * (at(1, 0, 1) - at(0, 0, 1));
    const double c11 = at(0, 1, 1) + f[0] * (at(1, 1, 1) - at(0, 1, 1));
    const double c0 = c00 + f[1] * (c10 - c00), c1 = c01 + f[1] * (c11 - c01);
    return c0 + f[2] * (c1 - c0);
}

__device__ inline void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// D at every (element, qp): diffusion w k adj(J) adj(J)^T / det J (rows of adj(J) are the
// cross products of the Jacobian columns), mass w k det J.  Layout [e][comp][qp].
__global__ void k_setup_qdata(int64_t nelem, int q, int ops, int ncomp, const double *__restrict__ vert,
                              const int32_t *__restrict__ hex, const DevTables *__restrict__ tab, CoeffDev cf,
                              double *__restrict__ qd, int *__restrict__ bad)
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
    const double col0[3] = {J[0][0], J[1][0], J[2][0]};
    const double col1[3] = {J[0][1], J[1][1], J[2][1]};
    const double col2[3] = {J[0][2], J[1][2], J[2][2]};
    double R0[3], R1[3], R2[3];
    cross(col1, col2, R0);
    cross(col2, col0, R1);
    cross(col0, col1, R2);
    const double det = col0[0] * R0[0] + col0[1] * R0[1] + col0[2] * R0[2];
    if (!(det > 0.0)) *bad = 1;
    const double wk = tab->w[a] * tab->w[b] * tab->w[c] * coeff_eval(cf, x);
    double *out = qd + e * (int64_t)ncomp * q3 + r;
    int comp = 0;
    if (ops & PA_DIFFUSION) {
        const double s = wk / det;
        auto dot = [](const double *u, const double *v) { return u[0] * v[0] + u[1] * v[1] + u[2] * v[2]; };
        out[0 * q3] = s * dot(R0, R0);
        out[1 * q3] = s * dot(R0, R1);
        out[2 * q3] = s * dot(R0, R2);
        out[3 * q3] = s * dot(R1, R1);
        out[4 * q3] = s * dot(R1, R2);
        out[5 * q3] = s * dot(R2, R2);
        comp = 6;
    }
    if (ops & PA_MASS) out[comp * q3] = wk * det;
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
    hipLaunchKernelGGL(k_setup_qdata, dim3(nblk(n)), dim3(256), 0, s, (int64_t)op->nelem, op->q, op->ops, op->ncomp,
                       op->d_vert, op->d_hex, op->d_tab, cf, op->d_qdata, d_bad);
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
