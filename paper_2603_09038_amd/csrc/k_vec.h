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

hipError_t vec_recip(double *y, const double *x, int64_t n, hipStream_t s);
hipError_t vec_dot(const double *x, const double *y, int64_t n, double *partial, double *out, hipStream_t s);

// r = b - r_in (r holds A x on entry), p = dinv r, scalars rz = r.dinv r, hist[0] = r.r
hipError_t cg_init(const double *b, double *r, double *p, const double *dinv, int64_t n, double *partial,
                   CgScalars *sc, double *hist, hipStream_t s);
// alpha = rz / (p . Ap)
hipError_t cg_alpha(const double *p, const double *Ap, int64_t n, double *partial, CgScalars *sc, hipStream_t s);
// x += alpha p, r -= alpha Ap, beta, p = dinv r + beta p; hist[2 it] = r.r, hist[2 it + 1] = breakdown flag
hipError_t cg_update(double *x, double *r, double *p, const double *Ap, const double *dinv, int64_t n,
                     double *partial, CgScalars *sc, double *hist, int it, hipStream_t s);

}  // namespace hexpa
