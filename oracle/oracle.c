/*
 * CPU FP64 oracle for the H1 mass and diffusion operators on trilinear hexahedra, and
 * for the mixed H1 x L2 gradient / divergence blocks of the acoustic operator (eq. (4)).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code with the HIP path.
 *
 * What it computes: the plain definition of the finite-element operator
 * A = G^T B^T D B G (the paper's operator decomposition, eq. (1), with the
 * parallel restriction P = I on one device), with B and D expanded to what they
 * stand for: at every Gauss point of every element the full 3-D basis values
 * phi_I and physical gradients grad phi_I = J^{-T} grad_ref phi_I are evaluated
 * by direct loops over all local nodes I = (i,j,k), and the dense element matrix
 *     A_e[I][J] = sum_q w_q kappa(x_q) detJ_q ( phi_I phi_J  [mass]
 *                                             + grad phi_I . grad phi_J [diffusion] )
 * is accumulated.  No sum factorization, no tensor-product contraction, no
 * quadrature-point data array: the factorized form of eq. (2) is what the HIP
 * path computes, and this is what it must equal up to rounding.
 *
 * Conventions (readings of points the paper leaves open):
 *  - reference element [0,1]^3, local node I = i + d j + d^2 k (i fastest), d = p+1;
 *  - nodes: Gauss-Lobatto-Legendre points; quadrature: q-point Gauss-Legendre per axis;
 *  - hex corner c = a + 2b + 4c' sits at reference vertex (a, b, c');
 *  - structured n^3 box: element e = ex + n ey + n^2 ez, global DOF of lattice node
 *    (I,J,K) = (ex p + i, ey p + j, ez p + k) is I + M J + M^2 K with M = n p + 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MASS 1
#define ORC_DIFFUSION 2

enum { ORC_COEFF_CONST = 0, ORC_COEFF_SINE = 1, ORC_COEFF_GRID = 2 };

typedef struct {
    int32_t kind;
    double value, amp, freq;
    const double *grid; /* [gz][gy][gx] over [0,1]^3, x fastest */
    int32_t gx, gy, gz;
} orc_coeff;

/* ------------------------------------------------------------------ 1-D */

/* Legendre P_n(t) and P_n'(t) on [-1,1] by the Bonnet recurrence. */
static void legendre(int n, double t, double *P, double *dP)
{
    double p0 = 1.0, p1 = t;
    if (n == 0) { *P = 1.0; *dP = 0.0; return; }
    for (int k = 2; k <= n; ++k) {
        double p2 = ((2.0 * k - 1.0) * t * p1 - (k - 1.0) * p0) / k;
        p0 = p1; p1 = p2;
    }
    *P = p1;
    /* P_n' = n (t P_n - P_{n-1}) / (t^2 - 1), valid away from +-1 */
    *dP = n * (t * p1 - p0) / (t * t - 1.0);
}

/* Locate all roots of f in (-1,1) by a sign-change scan followed by bisection. */
static int bisect_roots(double (*f)(int, double), int n, int expect, double *roots)
{
    const int S = 40000;
    int found = 0;
    double a = -1.0 + 1e-9, fa = f(n, a);
    for (int s = 1; s <= S && found < expect; ++s) {
        double b = -1.0 + 2.0 * s / S - (s == S ? 1e-9 : 0.0), fb = f(n, b);
        if (fa == 0.0) { roots[found++] = a; }
        else if (fa * fb < 0.0) {
            double lo = a, hi = b, flo = fa;
            for (int it = 0; it < 200; ++it) {
                double mid = 0.5 * (lo + hi), fm = f(n, mid);
                if (mid == lo || mid == hi) break;
                if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
            }
            roots[found++] = 0.5 * (lo + hi);
        }
        a = b; fa = fb;
    }
    return found;
}

static double leg_value(int n, double t) { double P, dP; legendre(n, t, &P, &dP); return P; }
static double leg_deriv(int n, double t) { double P, dP; legendre(n, t, &P, &dP); return dP; }

/* q-point Gauss-Legendre rule on [0,1]: points ascending, weights summing to 1. */
int orc_gauss(int q, double *x, double *w)
{
    double t[64];
    if (q < 1 || q > 64) return -1;
    if (bisect_roots(leg_value, q, q, t) != q) return -2;
    for (int i = 0; i < q; ++i) {
        double dP = leg_deriv(q, t[i]);
        x[i] = 0.5 * (t[i] + 1.0);
        w[i] = 0.5 * 2.0 / ((1.0 - t[i] * t[i]) * dP * dP);
    }
    return 0;
}

/* p+1 Gauss-Lobatto-Legendre nodes on [0,1]: 0, roots of P_p' mapped, 1. */
static double legd_fn(int n, double t) { return leg_deriv(n, t); }
int orc_gll(int p, double *x)
{
    double t[64];
    if (p < 1 || p > 63) return -1;
    x[0] = 0.0; x[p] = 1.0;
    if (p > 1) {
        if (bisect_roots(legd_fn, p, p - 1, t) != p - 1) return -2;
        for (int i = 0; i < p - 1; ++i) x[i + 1] = 0.5 * (t[i] + 1.0);
    }
    return 0;
}

/* All n Lagrange polynomials on the nodes and their derivatives at t (product formula). */
void orc_lagrange(int n, const double *nodes, double t, double *l, double *dl)
{
    for (int i = 0; i < n; ++i) {
        double v = 1.0, dv = 0.0;
        for (int m = 0; m < n; ++m) {
            if (m == i) continue;
            double den = nodes[i] - nodes[m];
            /* product rule: d/dt [v * (t - x_m)/den] */
            dv = dv * (t - nodes[m]) / den + v / den;
            v = v * (t - nodes[m]) / den;
        }
        l[i] = v;
        if (dl) dl[i] = dv;
    }
}

/* ------------------------------------------------------------ maps */

void orc_box_elem_dofs(int n, int p, int32_t *elem_dofs)
{
    const int d = p + 1;
    const int64_t M = (int64_t)n * p + 1;
    for (int ez = 0; ez < n; ++ez)
        for (int ey = 0; ey < n; ++ey)
            for (int ex = 0; ex < n; ++ex) {
                int64_t e = ex + (int64_t)n * (ey + (int64_t)n * ez);
                for (int k = 0; k < d; ++k)
                    for (int j = 0; j < d; ++j)
                        for (int i = 0; i < d; ++i) {
                            int64_t I = (int64_t)ex * p + i, J = (int64_t)ey * p + j, K = (int64_t)ez * p + k;
                            elem_dofs[e * d * d * d + i + d * (j + d * k)] = (int32_t)(I + M * (J + M * K));
                        }
            }
}

void orc_box_boundary(int n, int p, uint8_t *marker)
{
    const int64_t M = (int64_t)n * p + 1;
    for (int64_t K = 0; K < M; ++K)
        for (int64_t J = 0; J < M; ++J)
            for (int64_t I = 0; I < M; ++I)
                marker[I + M * (J + M * K)] =
                    (I == 0 || J == 0 || K == 0 || I == M - 1 || J == M - 1 || K == M - 1) ? 1 : 0;
}

/* -------------------------------------------------------- geometry */

/* Trilinear map x(xi) = sum_c X_c N_c(xi) and its Jacobian J[r][s] = d x_r / d xi_s. */
static void trilinear(const double *X /*[8][3]*/, const double xi[3], double x[3], double J[3][3])
{
    memset(J, 0, 9 * sizeof(double));
    x[0] = x[1] = x[2] = 0.0;
    for (int c = 0; c < 8; ++c) {
        int bit[3] = {c & 1, (c >> 1) & 1, (c >> 2) & 1};
        double f[3], df[3];
        for (int s = 0; s < 3; ++s) {
            f[s] = bit[s] ? xi[s] : 1.0 - xi[s];
            df[s] = bit[s] ? 1.0 : -1.0;
        }
        double N = f[0] * f[1] * f[2];
        double dN[3] = {df[0] * f[1] * f[2], f[0] * df[1] * f[2], f[0] * f[1] * df[2]};
        for (int r = 0; r < 3; ++r) {
            x[r] += X[3 * c + r] * N;
            for (int s = 0; s < 3; ++s) J[r][s] += X[3 * c + r] * dN[s];
        }
    }
}

/* det J and J^{-1} by cofactors. */
static double invert3(const double J[3][3], double Ji[3][3])
{
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    return det;
}

static double coeff_at(const orc_coeff *c, const double x[3])
{
    if (c->kind == ORC_COEFF_CONST) return c->value;
    if (c->kind == ORC_COEFF_SINE) {
        double w = c->freq * M_PI;
        return c->value + c->amp * sin(w * x[0]) * sin(w * x[1]) * sin(w * x[2]);
    }
    /* ORC_COEFF_GRID: trilinear interpolation of grid values on [0,1]^3 */
    int g[3] = {c->gx, c->gy, c->gz};
    int i0[3]; double fr[3];
    for (int s = 0; s < 3; ++s) {
        double t = x[s] < 0.0 ? 0.0 : (x[s] > 1.0 ? 1.0 : x[s]);
        t *= (g[s] - 1);
        int i = (int)floor(t);
        if (i > g[s] - 2) i = g[s] - 2;
        i0[s] = i; fr[s] = t - i;
    }
    double v = 0.0;
    for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
            for (int cx = 0; cx < 2; ++cx) {
                double wgt = (cx ? fr[0] : 1 - fr[0]) * (cy ? fr[1] : 1 - fr[1]) * (cz ? fr[2] : 1 - fr[2]);
                v += wgt * c->grid[(int64_t)(i0[0] + cx) + (int64_t)g[0] * ((i0[1] + cy) + (int64_t)g[1] * (i0[2] + cz))];
            }
    return v;
}

static void gather_corners(const double *vert, const int32_t *hex, int64_t e, double X[24])
{
    for (int c = 0; c < 8; ++c)
        for (int r = 0; r < 3; ++r) X[3 * c + r] = vert[3 * (int64_t)hex[8 * e + c] + r];
}

/* Per-element quadrature context: 1-D tables shared by all elements. */
typedef struct {
    int p, d, q, nd, nq;
    double nodes[64], qx[64], qw[64];
    double *L, *dL; /* [q][d] Lagrange values / derivatives at the Gauss points */
} tables;

static int tables_init(tables *T, int p, int q)
{
    T->p = p; T->d = p + 1; T->q = q; T->nd = T->d * T->d * T->d; T->nq = q * q * q;
    if (orc_gll(p, T->nodes) || orc_gauss(q, T->qx, T->qw)) return -1;
    T->L = (double *)malloc(sizeof(double) * q * T->d);
    T->dL = (double *)malloc(sizeof(double) * q * T->d);
    for (int a = 0; a < q; ++a) orc_lagrange(T->d, T->nodes, T->qx[a], T->L + a * T->d, T->dL + a * T->d);
    return 0;
}
static void tables_free(tables *T) { free(T->L); free(T->dL); }

/* Values and physical gradients of all d^3 basis functions at Gauss point (a,b,c);
   returns w * detJ and sets x (physical point). */
static double basis_at_qp(const tables *T, const double X[24], int a, int b, int c,
                          double *phi, double *gphi /*[nd][3]*/, double x[3], double *detJ_out)
{
    const int d = T->d;
    double xi[3] = {T->qx[a], T->qx[b], T->qx[c]};
    double J[3][3], Ji[3][3];
    trilinear(X, xi, x, J);
    double det = invert3(J, Ji);
    const double *La = T->L + a * d, *Lb = T->L + b * d, *Lc = T->L + c * d;
    const double *dLa = T->dL + a * d, *dLb = T->dL + b * d, *dLc = T->dL + c * d;
    for (int k = 0; k < d; ++k)
        for (int j = 0; j < d; ++j)
            for (int i = 0; i < d; ++i) {
                int I = i + d * (j + d * k);
                double gr[3] = {dLa[i] * Lb[j] * Lc[k], La[i] * dLb[j] * Lc[k], La[i] * Lb[j] * dLc[k]};
                phi[I] = La[i] * Lb[j] * Lc[k];
                for (int r = 0; r < 3; ++r) /* (grad phi)_r = sum_s (J^{-1})_{s r} (grad_ref phi)_s */
                    gphi[3 * I + r] = Ji[0][r] * gr[0] + Ji[1][r] * gr[1] + Ji[2][r] * gr[2];
            }
    if (detJ_out) *detJ_out = det;
    return T->qw[a] * T->qw[b] * T->qw[c] * det;
}

/* Dense element matrix by quadrature loops.  Returns min detJ over the Gauss points. */
static double elem_matrix(const tables *T, const double X[24], const orc_coeff *cf, int ops,
                          double *Ae, double *phi, double *gphi)
{
    const int nd = T->nd, q = T->q;
    double mindet = INFINITY;
    memset(Ae, 0, sizeof(double) * nd * nd);
    for (int c = 0; c < q; ++c)
        for (int b = 0; b < q; ++b)
            for (int a = 0; a < q; ++a) {
                double x[3], det;
                double wdet = basis_at_qp(T, X, a, b, c, phi, gphi, x, &det);
                if (det < mindet) mindet = det;
                double s = wdet * coeff_at(cf, x);
                for (int I = 0; I < nd; ++I)
                    for (int Jn = 0; Jn < nd; ++Jn) {
                        double v = 0.0;
                        if (ops & ORC_MASS) v += phi[I] * phi[Jn];
                        if (ops & ORC_DIFFUSION)
                            v += gphi[3 * I] * gphi[3 * Jn] + gphi[3 * I + 1] * gphi[3 * Jn + 1] + gphi[3 * I + 2] * gphi[3 * Jn + 2];
                        Ae[(int64_t)I * nd + Jn] += s * v;
                    }
            }
    return mindet;
}

/* ------------------------------------------------------ exported ops */

/* Dense element matrices for a list of elements (all if subset == NULL). */
int orc_elem_matrices(int64_t nsel, const int32_t *subset, const double *vert, const int32_t *hex,
                      int p, int q, const orc_coeff *cf, int ops, double *Ae_out, double *mindet_out)
{
    tables T;
    if (tables_init(&T, p, q)) return -1;
    const int nd = T.nd;
    double gmin = INFINITY;
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * nd);
        double *gphi = (double *)malloc(sizeof(double) * 3 * nd);
        double lmin = INFINITY;
#pragma omp for schedule(dynamic, 4)
        for (int64_t s = 0; s < nsel; ++s) {
            int64_t e = subset ? subset[s] : s;
            double X[24];
            gather_corners(vert, hex, e, X);
            double m = elem_matrix(&T, X, cf, ops, Ae_out + s * (int64_t)nd * nd, phi, gphi);
            if (m < lmin) lmin = m;
        }
#pragma omp critical
        if (lmin < gmin) gmin = lmin;
        free(phi); free(gphi);
    }
    if (mindet_out) *mindet_out = gmin;
    tables_free(&T);
    return 0;
}

/* y = sum_e G_e^T A_e G_e x with element matrices assembled on the fly.
   With subset != NULL only the listed elements contribute (used for timing samples). */
int orc_apply(int64_t nelem, const int64_t nsel, const int32_t *subset, const double *vert,
              const int32_t *hex, const int32_t *elem_dofs, int p, int q, const orc_coeff *cf, int ops,
              int64_t ndof, const double *x, double *y)
{
    tables T;
    if (tables_init(&T, p, q)) return -1;
    const int nd = T.nd;
    int64_t cnt = subset ? nsel : nelem;
    double *yE = (double *)malloc(sizeof(double) * cnt * nd);
    if (!yE) { tables_free(&T); return -3; }
#pragma omp parallel
    {
        double *Ae = (double *)malloc(sizeof(double) * nd * nd);
        double *phi = (double *)malloc(sizeof(double) * nd);
        double *gphi = (double *)malloc(sizeof(double) * 3 * nd);
        double *xE = (double *)malloc(sizeof(double) * nd);
#pragma omp for schedule(dynamic, 4)
        for (int64_t s = 0; s < cnt; ++s) {
            int64_t e = subset ? subset[s] : s;
            double X[24];
            gather_corners(vert, hex, e, X);
            elem_matrix(&T, X, cf, ops, Ae, phi, gphi);
            for (int I = 0; I < nd; ++I) xE[I] = x[elem_dofs[e * nd + I]];
            for (int I = 0; I < nd; ++I) {
                double acc = 0.0;
                for (int Jn = 0; Jn < nd; ++Jn) acc += Ae[(int64_t)I * nd + Jn] * xE[Jn];
                yE[s * nd + I] = acc;
            }
        }
        free(Ae); free(phi); free(gphi); free(xE);
    }
    memset(y, 0, sizeof(double) * ndof);
    for (int64_t s = 0; s < cnt; ++s) {
        int64_t e = subset ? subset[s] : s;
        for (int I = 0; I < nd; ++I) y[elem_dofs[e * nd + I]] += yE[s * nd + I];
    }
    free(yE);
    tables_free(&T);
    return 0;
}

/* y = sum_e G_e^T A_e G_e x with precomputed element matrices. */
void orc_apply_assembled(int64_t nelem, int nd, const double *Ae, const int32_t *elem_dofs,
                         int64_t ndof, const double *x, double *y)
{
    memset(y, 0, sizeof(double) * ndof);
    for (int64_t e = 0; e < nelem; ++e) {
        const double *A = Ae + e * (int64_t)nd * nd;
        const int32_t *g = elem_dofs + e * nd;
        for (int I = 0; I < nd; ++I) {
            double acc = 0.0;
            for (int Jn = 0; Jn < nd; ++Jn) acc += A[(int64_t)I * nd + Jn] * x[g[Jn]];
            y[g[I]] += acc;
        }
    }
}

/* diag(A)_i = sum_e (A_e)_{II} with I the local index of DOF i in element e. */
int orc_diag(int64_t nelem, const double *vert, const int32_t *hex, const int32_t *elem_dofs,
             int p, int q, const orc_coeff *cf, int ops, int64_t ndof, double *diag)
{
    tables T;
    if (tables_init(&T, p, q)) return -1;
    const int nd = T.nd;
    double *dE = (double *)malloc(sizeof(double) * nelem * nd);
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * nd);
        double *gphi = (double *)malloc(sizeof(double) * 3 * nd);
#pragma omp for schedule(dynamic, 4)
        for (int64_t e = 0; e < nelem; ++e) {
            double X[24];
            gather_corners(vert, hex, e, X);
            double *de = dE + e * nd;
            for (int I = 0; I < nd; ++I) de[I] = 0.0;
            for (int c = 0; c < q; ++c)
                for (int b = 0; b < q; ++b)
                    for (int a = 0; a < q; ++a) {
                        double x[3];
                        double s = basis_at_qp(&T, X, a, b, c, phi, gphi, x, NULL) * coeff_at(cf, x);
                        for (int I = 0; I < nd; ++I) {
                            double v = 0.0;
                            if (ops & ORC_MASS) v += phi[I] * phi[I];
                            if (ops & ORC_DIFFUSION)
                                v += gphi[3 * I] * gphi[3 * I] + gphi[3 * I + 1] * gphi[3 * I + 1] + gphi[3 * I + 2] * gphi[3 * I + 2];
                            de[I] += s * v;
                        }
                    }
        }
        free(phi); free(gphi);
    }
    memset(diag, 0, sizeof(double) * ndof);
    for (int64_t e = 0; e < nelem; ++e)
        for (int I = 0; I < nd; ++I) diag[elem_dofs[e * nd + I]] += dE[e * nd + I];
    free(dE);
    tables_free(&T);
    return 0;
}

/* Row-sampled apply: for each (element, local row) pair, the element's contribution
   a_e(phi_I, u_h) = sum_q w kappa detJ (phi_I u_h [mass] + grad phi_I . grad u_h [diff])
   with u_h = sum_J x_{G(e,J)} phi_J; contributions of pairs sharing an output row are
   summed into out[row_of_pair]. */
int orc_apply_rows(int64_t npairs, const int32_t *pair_elem, const int32_t *pair_local,
                   const int32_t *pair_out, int64_t nout, const double *vert, const int32_t *hex,
                   const int32_t *elem_dofs, int p, int q, const orc_coeff *cf, int ops,
                   const double *x, double *out)
{
    tables T;
    if (tables_init(&T, p, q)) return -1;
    const int nd = T.nd;
    double *contrib = (double *)malloc(sizeof(double) * (npairs > 0 ? npairs : 1));
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * nd);
        double *gphi = (double *)malloc(sizeof(double) * 3 * nd);
#pragma omp for schedule(dynamic, 1)
        for (int64_t s = 0; s < npairs; ++s) {
            int64_t e = pair_elem[s];
            int I = pair_local[s];
            double X[24];
            gather_corners(vert, hex, e, X);
            double acc = 0.0;
            for (int c = 0; c < q; ++c)
                for (int b = 0; b < q; ++b)
                    for (int a = 0; a < q; ++a) {
                        double xq[3];
                        double sc = basis_at_qp(&T, X, a, b, c, phi, gphi, xq, NULL) * coeff_at(cf, xq);
                        double u = 0.0, gu[3] = {0.0, 0.0, 0.0};
                        for (int Jn = 0; Jn < nd; ++Jn) {
                            double xv = x[elem_dofs[e * nd + Jn]];
                            u += xv * phi[Jn];
                            for (int r = 0; r < 3; ++r) gu[r] += xv * gphi[3 * Jn + r];
                        }
                        double v = 0.0;
                        if (ops & ORC_MASS) v += phi[I] * u;
                        if (ops & ORC_DIFFUSION) v += gphi[3 * I] * gu[0] + gphi[3 * I + 1] * gu[1] + gphi[3 * I + 2] * gu[2];
                        acc += sc * v;
                    }
            contrib[s] = acc;
        }
        free(phi); free(gphi);
    }
    memset(out, 0, sizeof(double) * nout);
    for (int64_t s = 0; s < npairs; ++s) out[pair_out[s]] += contrib[s];
    free(contrib);
    tables_free(&T);
    return 0;
}

/* Physical coordinates of the Gauss points, out[e][c][b][a][3] (a fastest). */
int orc_qpoints(int64_t nelem, const double *vert, const int32_t *hex, int q, double *out)
{
    double qx[64], qw[64];
    if (orc_gauss(q, qx, qw)) return -1;
#pragma omp parallel for
    for (int64_t e = 0; e < nelem; ++e) {
        double X[24], J[3][3];
        gather_corners(vert, hex, e, X);
        for (int c = 0; c < q; ++c)
            for (int b = 0; b < q; ++b)
                for (int a = 0; a < q; ++a) {
                    double xi[3] = {qx[a], qx[b], qx[c]};
                    trilinear(X, xi, out + 3 * (e * q * q * q + a + q * (b + q * c)), J);
                }
    }
    return 0;
}

/* Physical coordinates of every DOF node (GLL lattice mapped by its element). */
int orc_nodes(int64_t nelem, const double *vert, const int32_t *hex, const int32_t *elem_dofs,
              int p, double *out /*[ndof][3]*/)
{
    double nodes[64];
    const int d = p + 1, nd = d * d * d;
    if (orc_gll(p, nodes)) return -1;
    for (int64_t e = 0; e < nelem; ++e) {
        double X[24], J[3][3];
        gather_corners(vert, hex, e, X);
        for (int k = 0; k < d; ++k)
            for (int j = 0; j < d; ++j)
                for (int i = 0; i < d; ++i) {
                    double xi[3] = {nodes[i], nodes[j], nodes[k]};
                    trilinear(X, xi, out + 3 * (int64_t)elem_dofs[e * nd + i + d * (j + d * k)], J);
                }
    }
    return 0;
}

/* Load vector b_i = sum_e sum_q w detJ f_q phi_I(x_q), f given at the Gauss points [e][q^3]. */
int orc_load(int64_t nelem, const double *vert, const int32_t *hex, const int32_t *elem_dofs,
             int p, int q, const double *fq, int64_t ndof, double *b)
{
    tables T;
    if (tables_init(&T, p, q)) return -1;
    const int nd = T.nd, nq = T.nq;
    double *bE = (double *)malloc(sizeof(double) * nelem * nd);
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * nd);
        double *gphi = (double *)malloc(sizeof(double) * 3 * nd);
#pragma omp for
        for (int64_t e = 0; e < nelem; ++e) {
            double X[24];
            gather_corners(vert, hex, e, X);
            double *be = bE + e * nd;
            for (int I = 0; I < nd; ++I) be[I] = 0.0;
            for (int c = 0; c < q; ++c)
                for (int b = 0; b < q; ++b)
                    for (int a = 0; a < q; ++a) {
                        double x[3];
                        double s = basis_at_qp(&T, X, a, b, c, phi, gphi, x, NULL) * fq[e * nq + a + q * (b + q * c)];
                        for (int I = 0; I < nd; ++I) be[I] += s * phi[I];
                    }
        }
        free(phi); free(gphi);
    }
    memset(b, 0, sizeof(double) * ndof);
    for (int64_t e = 0; e < nelem; ++e)
        for (int I = 0; I < nd; ++I) b[elem_dofs[e * nd + I]] += bE[e * nd + I];
    free(bE);
    tables_free(&T);
    return 0;
}

/* ------------------------------------------- mixed H1 x L2 gradient block (acoustic operator)

   The off-diagonal blocks of the paper's block operator, eq. (4), for pressure p in the
   continuous order-p space (GLL nodes, global DOF map) and velocity u in the discontinuous
   order-pu space (Lagrange on the pu+1 Gauss-Legendre points per axis, element-local,
   three scalar components): with psi_J the velocity basis and phi_I the pressure basis,

       G_e[(c, J)][I] = (d phi_I / d x_c, psi_J)_e = sum_q w_q detJ_q psi_J(x_q) (J^{-T} grad_ref phi_I)_c

   so that (grad p, tau) = G p and -(u, grad v) = -G^T u.  The element matrices are built by
   plain quadrature loops with physical gradients (no sum factorization).  Velocity vectors
   are [nelem][3][nu], nu = (pu+1)^3, local node J = j1 + du (j2 + du j3), du = pu + 1. */

typedef struct {
    int du, nu;
    double nodes[64];
    double *L; /* [q][du] velocity basis values at the Gauss points */
} utables;

static int utables_init(utables *U, int pu, int q, const double *qx)
{
    double w[64];
    U->du = pu + 1;
    U->nu = U->du * U->du * U->du;
    if (orc_gauss(U->du, U->nodes, w)) return -1;
    U->L = (double *)malloc(sizeof(double) * q * U->du);
    for (int a = 0; a < q; ++a) orc_lagrange(U->du, U->nodes, qx[a], U->L + a * U->du, NULL);
    return 0;
}

static void mixed_elem(const tables *T, const utables *U, const double X[24], double *Ge, double *phi, double *gphi)
{
    const int nd = T->nd, nu = U->nu, du = U->du, q = T->q;
    memset(Ge, 0, sizeof(double) * 3 * nu * nd);
    for (int c = 0; c < q; ++c)
        for (int b = 0; b < q; ++b)
            for (int a = 0; a < q; ++a) {
                double x[3];
                double wdet = basis_at_qp(T, X, a, b, c, phi, gphi, x, NULL);
                for (int j3 = 0; j3 < du; ++j3)
                    for (int j2 = 0; j2 < du; ++j2)
                        for (int j1 = 0; j1 < du; ++j1) {
                            int J = j1 + du * (j2 + du * j3);
                            double psi = U->L[a * du + j1] * U->L[b * du + j2] * U->L[c * du + j3];
                            for (int comp = 0; comp < 3; ++comp) {
                                double *row = Ge + (int64_t)(comp * nu + J) * nd;
                                for (int I = 0; I < nd; ++I) row[I] += wdet * psi * gphi[3 * I + comp];
                            }
                        }
            }
}

/* Element matrices G_e [nsel][3 nu][nd] of the listed elements (all if subset == NULL). */
int orc_mixed_elem_matrices(int64_t nsel, const int32_t *subset, const double *vert, const int32_t *hex,
                            int p, int pu, int q, double *Ge_out)
{
    tables T;
    utables U;
    if (tables_init(&T, p, q)) return -1;
    if (utables_init(&U, pu, q, T.qx)) { tables_free(&T); return -1; }
    const int nd = T.nd, nu = U.nu;
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * nd);
        double *gphi = (double *)malloc(sizeof(double) * 3 * nd);
#pragma omp for schedule(dynamic, 2)
        for (int64_t s = 0; s < nsel; ++s) {
            int64_t e = subset ? subset[s] : s;
            double X[24];
            gather_corners(vert, hex, e, X);
            mixed_elem(&T, &U, X, Ge_out + s * (int64_t)3 * nu * nd, phi, gphi);
        }
        free(phi); free(gphi);
    }
    free(U.L);
    tables_free(&T);
    return 0;
}

/* yu = G p (element-local velocity space) and yp = -G^T u (global pressure vector). */
int orc_mixed_apply(int64_t nelem, const double *vert, const int32_t *hex, const int32_t *elem_dofs, int p, int pu,
                    int q, int64_t ndof, const double *u, const double *pv, double *yu, double *yp)
{
    tables T;
    utables U;
    if (tables_init(&T, p, q)) return -1;
    if (utables_init(&U, pu, q, T.qx)) { tables_free(&T); return -1; }
    const int nd = T.nd, nu = U.nu;
    double *ypE = (double *)malloc(sizeof(double) * nelem * nd);
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * nd);
        double *gphi = (double *)malloc(sizeof(double) * 3 * nd);
        double *Ge = (double *)malloc(sizeof(double) * 3 * nu * nd);
#pragma omp for schedule(dynamic, 2)
        for (int64_t e = 0; e < nelem; ++e) {
            double X[24];
            gather_corners(vert, hex, e, X);
            mixed_elem(&T, &U, X, Ge, phi, gphi);
            const int32_t *g = elem_dofs + e * nd;
            for (int r = 0; r < 3 * nu; ++r) {
                double acc = 0.0;
                for (int I = 0; I < nd; ++I) acc += Ge[(int64_t)r * nd + I] * pv[g[I]];
                yu[e * 3 * nu + r] = acc;
            }
            for (int I = 0; I < nd; ++I) {
                double acc = 0.0;
                for (int r = 0; r < 3 * nu; ++r) acc += Ge[(int64_t)r * nd + I] * u[e * 3 * nu + r];
                ypE[e * nd + I] = -acc;
            }
        }
        free(phi); free(gphi); free(Ge);
    }
    memset(yp, 0, sizeof(double) * ndof);
    for (int64_t e = 0; e < nelem; ++e)
        for (int I = 0; I < nd; ++I) yp[elem_dofs[e * nd + I]] += ypE[e * nd + I];
    free(ypE);
    free(U.L);
    tables_free(&T);
    return 0;
}

/* Row-sum lumped masses: mu[e][J] = sum_q w detJ rho psi_J (the same for each velocity
   component), mp[i] = sum_e sum_q w detJ phi_I / bulk (assembled). */
int orc_mixed_lumped(int64_t nelem, const double *vert, const int32_t *hex, const int32_t *elem_dofs, int p, int pu,
                     int q, double rho, double bulk, int64_t ndof, double *mu, double *mp)
{
    tables T;
    utables U;
    if (tables_init(&T, p, q)) return -1;
    if (utables_init(&U, pu, q, T.qx)) { tables_free(&T); return -1; }
    const int nd = T.nd, nu = U.nu, du = U.du;
    double *mpE = (double *)malloc(sizeof(double) * nelem * nd);
#pragma omp parallel
    {
        double *phi = (double *)malloc(sizeof(double) * nd);
        double *gphi = (double *)malloc(sizeof(double) * 3 * nd);
#pragma omp for
        for (int64_t e = 0; e < nelem; ++e) {
            double X[24];
            gather_corners(vert, hex, e, X);
            for (int J = 0; J < nu; ++J) mu[e * nu + J] = 0.0;
            for (int I = 0; I < nd; ++I) mpE[e * nd + I] = 0.0;
            for (int c = 0; c < q; ++c)
                for (int b = 0; b < q; ++b)
                    for (int a = 0; a < q; ++a) {
                        double x[3];
                        double wdet = basis_at_qp(&T, X, a, b, c, phi, gphi, x, NULL);
                        for (int j3 = 0; j3 < du; ++j3)
                            for (int j2 = 0; j2 < du; ++j2)
                                for (int j1 = 0; j1 < du; ++j1)
                                    mu[e * nu + j1 + du * (j2 + du * j3)] +=
                                        wdet * rho * U.L[a * du + j1] * U.L[b * du + j2] * U.L[c * du + j3];
                        for (int I = 0; I < nd; ++I) mpE[e * nd + I] += wdet * phi[I] / bulk;
                    }
        }
        free(phi); free(gphi);
    }
    memset(mp, 0, sizeof(double) * ndof);
    for (int64_t e = 0; e < nelem; ++e)
        for (int I = 0; I < nd; ++I) mp[elem_dofs[e * nd + I]] += mpE[e * nd + I];
    free(mpE);
    free(U.L);
    tables_free(&T);
    return 0;
}

/* Coefficient kappa at arbitrary physical points xyz [n][3] (the same evaluation the
   element matrices use at the quadrature points). */
void orc_coeff_points(const orc_coeff *cf, int64_t n, const double *xyz, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = coeff_at(cf, xyz + 3 * i);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
