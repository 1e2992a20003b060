// Kernels of the learned preconditioner (k_nn.hip): the per-element convolutional
// network, its backward pass and Adam, the tile gather/averaged scatter, and the p=1
// coarse level (transfers, probed 27-point stencil, fixed-iteration Jacobi-PCG).
#pragma once
#include "internal.h"
#include "k_vec.h"

namespace hexpa {

constexpr int kNetCin = 2;       // input channels: normalised residual, log kappa
constexpr int kNetCh = 16;       // hidden channels
constexpr int kNetW1 = kNetCh * kNetCin * 27, kNetW2 = kNetCh * kNetCh * 27, kNetW3 = kNetCh * 27;
// flat parameter vector: W1 [16][2][27], b1 [16], W2 [16][16][27], b2 [16], W3 [1][16][27], b3 [1]
constexpr int kNetParams = kNetW1 + kNetCh + kNetW2 + kNetCh + kNetW3 + 1;
constexpr int kNetOffW1 = 0, kNetOffB1 = kNetW1, kNetOffW2 = kNetOffB1 + kNetCh, kNetOffB2 = kNetOffW2 + kNetW2,
              kNetOffW3 = kNetOffB2 + kNetCh, kNetOffB3 = kNetOffW3 + kNetW3;

// Floats of weight-gradient partial sums the backward pass needs.
int64_t nn_partial_floats();

// Tile edge n = p + 1 in {3, 4, 5}.  Activations [e][c][n^3].
// wt: kNetW1 + kNetW2 + kNetW3 floats of transposed weights.
hipError_t nn_forward(int n, int64_t nelem, const float *params, float *wt, const float *x0, float *a1, float *a2,
                      float *out, hipStream_t s);
// grads += dL/dparams given gout = dL/dout; ga1, ga2 are [e][16][n^3] work arrays,
// wt holds kNetW2 floats, partial nn_partial_floats().
hipError_t nn_backward(int n, int64_t nelem, const float *params, const float *x0, const float *a1, const float *a2,
                       const float *gout, float *ga2, float *ga1, float *grads, float *wt, float *partial,
                       hipStream_t s);
// Inference in one kernel with FP16 MFMA (FP32 accumulation): z += W G^T (s_e NN(...)).
// wpack: nn_pack16_bytes() of device scratch for the lane-ordered FP16 weights.
int64_t nn_pack16_bytes();
hipError_t nn_infer16(int n, int64_t nelem, const float *params, void *wpack, const double *r, const int32_t *emap,
                      const float *logk, const double *inv_mult, double scale, double *z, hipStream_t s);
// x0 tiles [2 nelem][2][n^3]: tile e = [G_e r / s_e, logk_e], tile nelem + e = [-G_e r / s_e,
// logk_e]; s_e = RMS of G_e r (1 where it vanishes).
hipError_t nn_input(int n, int64_t nelem, const double *r, const int32_t *emap, const float *logk, float *x0,
                    float *s, hipStream_t st);
// z[g] += scale s_e (out_e - out_{nelem+e}) / 2 inv_mult[g] over all element nodes (the odd part).
hipError_t nn_output(int n, int64_t nelem, const float *out, const float *s, const int32_t *emap,
                     const double *inv_mult, double scale, double *z, hipStream_t st);
// gout_e = s_e inv_mult[g] gz[g] / 2, gout_{nelem+e} = -gout_e (adjoint of nn_output).
hipError_t nn_output_grad(int n, int64_t nelem, const double *gz, const float *s, const int32_t *emap,
                          const double *inv_mult, float *gout, hipStream_t st);
// inv_mult[g] = 1 / (number of elements holding g).
hipError_t nn_inv_mult(int n, int64_t nelem, int64_t ndof, const int32_t *emap, double *inv_mult, hipStream_t s);
// Adam (beta1 0.9, beta2 0.999, eps 1e-8) on n parameters, step = 1, 2, ...; zeroes g.
hipError_t nn_adam(float *p, float *g, float *m, float *v, int n, double lr, int step, hipStream_t s);
hipError_t vec_fill_f32(float *y, float v, int64_t n, hipStream_t s);

// ------------------------------------------------------------------ coarse level
struct CoarseScalars {
    double rz, alpha, beta, pAp;
    unsigned int count;  // blocks finished in the current reduction (reset by the last one)
    int pad;
};
struct BoxDims {
    int nx, ny, nz, p;
};
// uf (+)= P1 u1: nodal interpolation of the p=1 field at the fine GLL nodes.
hipError_t coarse_prolong(const BoxDims &b, const double *gll, const double *u1, double *uf, bool add, hipStream_t s);
// r1 = P1^T rf (three separable 1-D passes, fixed summation order); t1, t2 are work arrays
// of (nx+1)(ny p+1)(nz p+1) and (nx+1)(ny+1)(nz p+1) values.
hipError_t coarse_restrict(const BoxDims &b, const double *gll, const double *rf, double *r1, double *t1, double *t2,
                           hipStream_t s);
// probe vector of class c in {0..26}: 1 where (I mod 3, J mod 3, K mod 3) == c
hipError_t coarse_probe_vec(const BoxDims &b, int cls, double *v, hipStream_t s);
// S[i][slot] = (A v_cls)[i] for the neighbour of i in class cls; constrained rows/columns.
hipError_t coarse_probe_gather(const BoxDims &b, int cls, const double *y, const uint8_t *ess1, double *S,
                               hipStream_t s);
hipError_t coarse_dinv(int64_t n1, const double *S, double *dinv, hipStream_t s);
// k fixed Jacobi-PCG iterations on S u = r1 from u = 0 (r1 is overwritten with the residual).
hipError_t coarse_pcg(const BoxDims &b, const double *S, const double *dinv, double *r1, double *u, double *z,
                      double *p0, double *p1, double *Ap, double *partial, CoarseScalars *sc, int iters,
                      hipStream_t s);

// vector helpers
// sc[0] = num, sc[1] = den on entry: g *= 2 / den, sc[2] = num / den
hipError_t vec_loss_scale(double *g, int64_t n, double *sc, hipStream_t s);
hipError_t vec_sub(double *y, const double *a, const double *b, int64_t n, hipStream_t s);  // y = a - b
hipError_t vec_mul(double *y, const double *a, const double *b, int64_t n, hipStream_t s);  // y = a * b

}  // namespace hexpa
