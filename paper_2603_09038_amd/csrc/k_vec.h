// Vector and CG kernels (k_vec.hip).
#pragma once
#include "internal.h"

namespace hexpa {

constexpr int kRedBlocks = 1024;  // fixed block count of every reduction: reproducible sums

struct CgScalars {
    double rz, rr, pAp, alpha, beta;
    double rz_prev;  // rz of the previous iteration (read by the direction update)
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
// alpha = rz / (p . Ap) into sc (for the FCG update)
template <class T>
hipError_t cg_alpha(const T *p, const T *Ap, int64_t n, double *partial, CgScalars *sc, hipStream_t s);

// One PCG iteration after y = A p is three kernels:
//   cg_pap        partial sums of p . Ap                                   -> pap_part
//   cg_update_xr  alpha = rz / (p . Ap) (breakdown if not > 0), x += alpha p, r -= alpha Ap,
//                 rz_prev = rz, partial sums of (r . dinv r, r . r)         -> rz_part
//   cg_update_dir beta = rz_new / (rz_prev f), rz = rz_new, p = dinv r + beta p, Ap = 0
//                 (when Ap_zero is given: the next apply accumulates into it);
//                 hist[2 it] = r.r, hist[2 it + 1] = breakdown flag
// pap_part and rz_part are separate arrays of kRedBlocks (x2) doubles.  cg_rz_partials
// writes rz_part for a given r (after a residual replacement); f is the factor by which r
// and p were rescaled since rz_prev was taken (1 if they were not).
template <class T>
hipError_t cg_pap(const T *p, const T *Ap, int64_t n, double *pap_part, hipStream_t s);
template <class T>
hipError_t cg_update_xr(T *x, T *r, const T *p, const T *Ap, const T *dinv, int64_t n, const double *pap_part,
                        double *rz_part, CgScalars *sc, hipStream_t s);
template <class T>
hipError_t cg_rz_partials(const T *r, const T *dinv, int64_t n, double *rz_part, hipStream_t s);
template <class T>
hipError_t cg_update_dir(T *p, const T *r, const T *dinv, T *Ap_zero, int64_t n, const double *rz_part, CgScalars *sc,
                         double *hist, int it, double f, hipStream_t s);

// ------------------------------------------------------------------ FCG vectors
// x += alpha p; rold = r; r -= alpha Ap; hist[2 it] = r.r, hist[2 it + 1] = breakdown
hipError_t fcg_update(double *x, double *r, double *rold, const double *p, const double *Ap, int64_t n,
                      double *partial, CgScalars *sc, double *hist, int it, hipStream_t s);
// beta = (z.(r - rold)) / rz, rz = z.r (rold == nullptr: beta = 0, first direction), p = z + beta p
hipError_t fcg_direction(const double *z, const double *r, const double *rold, double *p, int64_t n, double *partial,
                         CgScalars *sc, hipStream_t s);

}  // namespace hexpa
