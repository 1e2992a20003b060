// Vector and CG kernels (k_vec.hip).
#pragma once
#include "internal.h"

namespace hexpa {

constexpr int kRedBlocks = 1024;  // fixed block count of every reduction: reproducible sums

struct CgScalars {
    double rz, rr, pAp, alpha, beta;
    int breakdown;
    int pad;
};

hipError_t vec_fill(float *y, float v, int64_t n, hipStream_t s);
hipError_t vec_set_list(float *y, float v, const int32_t *list, int n, hipStream_t s);
hipError_t vec_recip(double *y, const double *x, int64_t n, hipStream_t s);
hipError_t vec_to_f32(float *y, const double *x, double scale, int64_t n, hipStream_t s);  // y = (float)(x*scale)
hipError_t vec_axpy_f32(double *x, double a, const float *d, int64_t n, hipStream_t s);    // x += a*d
hipError_t vec_maxabs(const double *x, int64_t n, double *partial, double *out, hipStream_t s);
template <class T>
hipError_t vec_dot(const T *x, const T *y, int64_t n, double *partial, double *out, hipStream_t s);

// r = b - r_in (r holds A x on entry; b == nullptr: r kept), p = dinv r,
// scalars rz = r.dinv r, hist[0] = r.r  (all sums in FP64)
template <class T>
hipError_t cg_init(const T *b, T *r, T *p, const T *dinv, int64_t n, double *partial, CgScalars *sc, double *hist,
                   hipStream_t s);
// alpha = rz / (p . Ap)
template <class T>
hipError_t cg_alpha(const T *p, const T *Ap, int64_t n, double *partial, CgScalars *sc, hipStream_t s);
// x += alpha p, r -= alpha Ap, beta, p = dinv r + beta p; hist[2 it] = r.r, hist[2 it + 1] = breakdown flag
template <class T>
hipError_t cg_update(T *x, T *r, T *p, const T *Ap, const T *dinv, int64_t n, double *partial, CgScalars *sc,
                     double *hist, int it, hipStream_t s);

// The two halves of cg_update, for solvers that act between them:
// x += alpha p, r -= alpha Ap, partial sums of (r . dinv r, r . r)
template <class T>
hipError_t cg_update_xr(T *x, T *r, const T *p, const T *Ap, const T *dinv, int64_t n, double *partial, CgScalars *sc,
                        hipStream_t s);
// the same partial sums for a given r (after it has been replaced)
template <class T>
hipError_t cg_rz_partials(const T *r, const T *dinv, int64_t n, double *partial, hipStream_t s);
// beta = rz_new / (rz f), rz = rz_new, p = dinv r + beta p; hist as cg_update.  f: factor by
// which r and p were rescaled since rz was taken (1 if they were not)
template <class T>
hipError_t cg_update_dir(T *p, const T *r, const T *dinv, int64_t n, double *partial, CgScalars *sc, double *hist,
                         int it, double f, hipStream_t s);

// ------------------------------------------------------------------ FCG vectors
// x += alpha p; rold = r; r -= alpha Ap; hist[2 it] = r.r, hist[2 it + 1] = breakdown
hipError_t fcg_update(double *x, double *r, double *rold, const double *p, const double *Ap, int64_t n,
                      double *partial, CgScalars *sc, double *hist, int it, hipStream_t s);
// beta = (z.(r - rold)) / rz, rz = z.r (rold == nullptr: beta = 0, first direction), p = z + beta p
hipError_t fcg_direction(const double *z, const double *r, const double *rold, double *p, int64_t n, double *partial,
                         CgScalars *sc, hipStream_t s);

}  // namespace hexpa
