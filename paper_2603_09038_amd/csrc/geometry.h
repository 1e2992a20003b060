// Geometry of trilinear hexahedra at quadrature points, shared by the setup kernels (which
// store D) and the matrix-free apply (which recomputes D in the D-step).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace hexpa {

// Trilinear geometry of one hexahedron: corner c = a + 2b + 4c' at reference vertex (a,b,c').
struct Hex {
    double X[8][3];
};

__device__ __forceinline__ void load_hex(const double *__restrict__ vert, const int32_t *__restrict__ hex, int64_t e, Hex &h)
{
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int64_t v = hex[e * 8 + c];
#pragma unroll
        for (int r = 0; r < 3; ++r) h.X[c][r] = vert[v * 3 + r];
    }
}

// Position and Jacobian columns: dx/dxi_s is the blend of the four edge vectors along s.
__device__ __forceinline__ void map_point(const Hex &h, double u, double v, double w, double x[3], double J[3][3])
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

__device__ __forceinline__ double coeff_eval(const CoeffDev &cf, const double x[3])
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

__device__ __forceinline__ void cross(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

// The D values of one quadrature point (reference coordinates u, v, w, weight wq): for
// diffusion w k adj(J) adj(J)^T / det J (rows of adj(J) are the cross products of the
// Jacobian columns; order 00, 01, 02, 11, 12, 22), then for mass w k det J.  Returns det J.
template <int OPS>
__device__ __forceinline__ double qp_data(const Hex &h, double u, double v, double w, double wq, const CoeffDev &cf,
                                          double *out)
{
    double x[3], J[3][3];
    map_point(h, u, v, w, x, J);
    const double col0[3] = {J[0][0], J[1][0], J[2][0]};
    const double col1[3] = {J[0][1], J[1][1], J[2][1]};
    const double col2[3] = {J[0][2], J[1][2], J[2][2]};
    double R0[3], R1[3], R2[3];
    cross(col1, col2, R0);
    cross(col2, col0, R1);
    cross(col0, col1, R2);
    const double det = col0[0] * R0[0] + col0[1] * R0[1] + col0[2] * R0[2];
    const double wk = wq * coeff_eval(cf, x);
    int comp = 0;
    if constexpr ((OPS & PA_DIFFUSION) != 0) {
        const double s = wk / det;
        auto dot = [](const double *p, const double *q) { return p[0] * q[0] + p[1] * q[1] + p[2] * q[2]; };
        out[0] = s * dot(R0, R0);
        out[1] = s * dot(R0, R1);
        out[2] = s * dot(R0, R2);
        out[3] = s * dot(R1, R1);
        out[4] = s * dot(R1, R2);
        out[5] = s * dot(R2, R2);
        comp = 6;
    }
    if constexpr ((OPS & PA_MASS) != 0) out[comp] = wk * det;
    return det;
}

}  // namespace hexpa
