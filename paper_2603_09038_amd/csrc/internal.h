// Internal declarations of the hexpa library (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/hexpa.h"

namespace hexpa {

constexpr int kMaxP = 8;
constexpr int kMaxD = kMaxP + 1;
constexpr int kMaxQ = kMaxP + 2;

// Thread-local error message for pa_last_error().
void set_error(const std::string &msg);

// 1-D tables (tables.cpp).
struct Tables1D {
    int p = 0, d = 0, q = 0;
    std::vector<double> nodes, qpts, qwts;  // GLL nodes [d], Gauss points/weights [q] on [0,1]
    std::vector<double> B, G;               // [q][d]: l_i(x_a), l_i'(x_a)
};
bool make_tables(int p, int q, Tables1D &t, std::string &err);
// Discontinuous (L2) space of order pu: Lagrange basis on the pu+1 Gauss-Legendre points,
// values (and derivatives) at the q Gauss points
bool make_l2_tables(int pu, int q, Tables1D &t, std::string &err);

// Device-side 1-D table block: B[q][d], G[q][d] packed (kMaxQ*kMaxD each).
struct DevTables {
    double B[kMaxQ * kMaxD];
    double G[kMaxQ * kMaxD];
    double w[kMaxQ];
    double x[kMaxQ];
    double nodes[kMaxD];
};

struct CoeffDev {
    int32_t kind;
    double value, amp, freq;
    const double *grid;  // device
    int32_t gx, gy, gz;
};

}  // namespace hexpa

struct pa_op {
    int p = 0, d = 0, q = 0, ops = 0, ncomp = 0;
    int nelem = 0, ndof = 0, ness = 0;
    int nx = 0, ny = 0, nz = 0;
    int variant = PA_VARIANT_MFMA;
    int grid_cap = 0;                // > 0: at most this many workgroups per apply launch (pa_set_grid_cap)
    int device = 0;
    int32_t *d_elem_dofs = nullptr;  // [nelem][d^3]
    double *d_qdata = nullptr;       // [nelem][ncomp][q^3]
    float *d_qdata32 = nullptr;      // FP32 copy of D for the mixed-precision apply (lazy)
    double *d_qbuf = nullptr;        // quadrature-point tensor of the unfused apply (lazy)
    double *d_vert = nullptr;        // [nvert][3]
    int32_t *d_hex = nullptr;        // [nelem][8]
    int nvert = 0;
    hexpa::DevTables *d_tab = nullptr;
    double *d_grid = nullptr;        // coefficient grid (device copy)
    hexpa::CoeffDev coeff{};         // coefficient as the kernels see it (grid -> d_grid)
    int32_t *d_ess = nullptr;        // [ness]
    // colour classes: elements of colour c are d_color_elems[color_off[c] .. color_off[c+1])
    int32_t *d_color_elems = nullptr;
    int color_off[9] = {0};
    // handle-owned scratch for constrained apply and solvers
    double *d_scratch = nullptr;
    size_t scratch_len = 0;
    hexpa::Tables1D tab;
};

namespace hexpa {
// Kernel launchers (implemented in the .hip files).
hipError_t launch_setup_qdata(const pa_op *op, const CoeffDev &cf, int *d_bad, hipStream_t s);
hipError_t launch_qpoints(const pa_op *op, double *xyz, hipStream_t s);
hipError_t launch_nodes(const pa_op *op, double *xyz, hipStream_t s);
// log kappa at every (element, local node) as FP32 [nelem][d^3]
hipError_t logk_tiles(const pa_op *op, float *out, hipStream_t s);
hipError_t launch_load(const pa_op *op, const double *fq, double *b, hipStream_t s);
// apply: y += A x over the listed elements (elem_list == nullptr: all); the unfused
// variants stage the quadrature-point tensor in qbuf (nullptr: the handle's d_qbuf)
hipError_t launch_apply(const pa_op *op, int variant, const double *x, double *y,
                        const int32_t *elem_list, int nlist, hipStream_t s, bool *supported,
                        double *qbuf = nullptr);
hipError_t launch_apply_lp(const pa_op *op, int fmt, const float *x, float *y, hipStream_t s, bool *supported);
hipError_t launch_diag(const pa_op *op, double *diag, hipStream_t s);
hipError_t launch_debug_mfma16(int bf, const float *A, const float *B, float *D, hipStream_t s);
hipError_t launch_debug_mfma(int shape, const double *A, const double *B, double *D, hipStream_t s);
// host-side operator actions (api.cpp): y = A x over all elements (y zeroed first unless
// zero_first is false), and y = A_c x with the essential rows/columns of the identity
int do_apply(pa_op *op, int variant, const double *x, double *y, hipStream_t s, bool zero_first = true);
int do_apply_constrained(pa_op *op, const double *x, double *y, hipStream_t s);
// learned preconditioner (learned.cpp): z = M(r) and the operator the handle is bound to
int lp_precondition(pa_lp *lp, const double *r, double *z, hipStream_t s);
pa_op *lp_operator(const pa_lp *lp);
// vector kernels (k_vec.hip)
hipError_t vec_fill(double *y, double v, int64_t n, hipStream_t s);
hipError_t vec_copy(double *y, const double *x, int64_t n, hipStream_t s);
hipError_t vec_zero_list(double *y, const int32_t *list, int n, hipStream_t s);
hipError_t vec_copy_list(double *y, const double *x, const int32_t *list, int n, hipStream_t s);
hipError_t vec_set_list(double *y, double v, const int32_t *list, int n, hipStream_t s);
}  // namespace hexpa
