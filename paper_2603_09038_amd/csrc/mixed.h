// Internal declarations of the mixed H1 x L2 operator (the paper's own acoustic operator).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hexpa {
constexpr int kMixLdsBudget = 48 * 1024;  // LDS bytes per workgroup of the fused mixed kernel
}  // namespace hexpa

struct pa_mixed {
    int p = 0, pu = 0, q = 0;
    int nelem = 0, ndof = 0, nvel = 0, nvert = 0;
    int device = 0, grid_cap = 0;
    double rho = 1.0, bulk = 1.0;
    int32_t *d_emap = nullptr;          // [nelem][(p+1)^3] pressure DOF map
    double *d_qdata = nullptr;          // [nelem][9][q^3]: E_cm = w adj(J)_mc
    double *d_vert = nullptr;           // [nvert][3]
    int32_t *d_hex = nullptr;           // [nelem][8]
    hexpa::DevTables *d_tabp = nullptr; // pressure basis (GLL nodes) at the Gauss points
    hexpa::DevTables *d_tabu = nullptr; // velocity basis (Gauss-Legendre nodes) at the Gauss points
    double *d_minv_u = nullptr;         // [nvel] inverse lumped velocity mass (RK4; made on first use)
    double *d_minv_p = nullptr;         // [ndof] inverse lumped pressure mass
    double *d_rk = nullptr;             // RK4 work: yu, acc_u, xs_u [nvel] and yp, acc_p, xs_p [ndof]
};

namespace hexpa {
bool mixed_supported(int p, int pu, int q);
int mixed_elems_per_group(int p, int pu, int q);
hipError_t launch_mixed(const pa_mixed *m, const double *u, const double *p, double *yu, double *yp, hipStream_t s);
hipError_t launch_mixed_qdata(const pa_mixed *m, int *bad, hipStream_t s);
hipError_t launch_mixed_lumped(const pa_mixed *m, double *mu, double *mp, hipStream_t s);
hipError_t launch_rk_stage(int64_t n, const double *y, const double *minv, double *x, double *acc, double *xs,
                           int first, double ca, double cx, int last, hipStream_t s);
}  // namespace hexpa
