// 1-D tables of the tensor-product basis (the B^{1d} factors of the paper's eq. (2)):
// Gauss-Lobatto-Legendre nodes, Gauss-Legendre points/weights on [0,1], and the Lagrange
// basis values B[a][i] = l_i(x_a) and derivatives G[a][i] = l_i'(x_a) at the Gauss points.
#include <cmath>

#include "internal.h"

namespace hexpa {

namespace {

// P_n(t), P_n'(t) on [-1,1] (three-term recurrence; derivative by the Legendre ODE-free
// relation built alongside the recurrence: P_k' = P_{k-2}' + (2k-1) P_{k-1}).
void legendre_pd(int n, double t, double &P, double &dP)
{
    double pm2 = 1.0, pm1 = t, dm2 = 0.0, dm1 = 1.0;
    if (n == 0) { P = 1.0; dP = 0.0; return; }
    if (n == 1) { P = t; dP = 1.0; return; }
    for (int k = 2; k <= n; ++k) {
        double pk = ((2.0 * k - 1.0) * t * pm1 - (k - 1.0) * pm2) / k;
        double dk = dm2 + (2.0 * k - 1.0) * pm1;
        pm2 = pm1; pm1 = pk; dm2 = dm1; dm1 = dk;
    }
    P = pm1; dP = dm1;
}

bool gauss_legendre(int q, std::vector<double> &x, std::vector<double> &w)
{
    x.assign(q, 0.0); w.assign(q, 0.0);
    for (int i = 0; i < q; ++i) {
        // Newton from the asymptotic guess; roots come out descending in t
        double t = std::cos(M_PI * (i + 0.75) / (q + 0.5));
        double P, dP;
        for (int it = 0; it < 100; ++it) {
            legendre_pd(q, t, P, dP);
            double dt = P / dP;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        legendre_pd(q, t, P, dP);
        x[q - 1 - i] = 0.5 * (1.0 + t);
        w[q - 1 - i] = 1.0 / ((1.0 - t * t) * dP * dP);  // 2/((1-t^2)P'^2) halved for [0,1]
    }
    return true;
}

bool gauss_lobatto(int p, std::vector<double> &x)
{
    x.assign(p + 1, 0.0);
    x[0] = 0.0; x[p] = 1.0;
    for (int i = 1; i < p; ++i) {
        // interior nodes: roots of P_p', Newton with P_p'' from the Legendre equation
        double t = -std::cos(M_PI * i / p);
        for (int it = 0; it < 100; ++it) {
            double P, dP;
            legendre_pd(p, t, P, dP);
            double d2P = (2.0 * t * dP - p * (p + 1.0) * P) / (1.0 - t * t);
            double dt = dP / d2P;
            t -= dt;
            if (std::fabs(dt) < 1e-17) break;
        }
        x[i] = 0.5 * (1.0 + t);
    }
    return true;
}

// Barycentric Lagrange interpolation on the nodes: values and derivatives at t.
void lagrange_bary(const std::vector<double> &xn, double t, double *l, double *dl)
{
    const int n = (int)xn.size();
    std::vector<double> wb(n);
    for (int i = 0; i < n; ++i) {
        double prod = 1.0;
        for (int m = 0; m < n; ++m)
            if (m != i) prod *= (xn[i] - xn[m]);
        wb[i] = 1.0 / prod;
    }
    int hit = -1;
    for (int i = 0; i < n; ++i)
        if (t == xn[i]) hit = i;
    if (hit >= 0) {
        for (int i = 0; i < n; ++i) {
            l[i] = (i == hit) ? 1.0 : 0.0;
            if (i != hit) {
                dl[i] = (wb[i] / wb[hit]) / (xn[hit] - xn[i]);
            } else {
                double s = 0.0;
                for (int m = 0; m < n; ++m)
                    if (m != hit) s += 1.0 / (xn[hit] - xn[m]);
                dl[i] = s;
            }
        }
        return;
    }
    double den = 0.0;
    for (int m = 0; m < n; ++m) den += wb[m] / (t - xn[m]);
    for (int i = 0; i < n; ++i) {
        l[i] = (wb[i] / (t - xn[i])) / den;
        double s = 0.0;
        for (int m = 0; m < n; ++m)
            if (m != i) s += 1.0 / (t - xn[m]);
        dl[i] = l[i] * s;
    }
}

}  // namespace

bool make_tables(int p, int q, Tables1D &t, std::string &err)
{
    if (p < 1 || p > kMaxP || q < 1 || q > kMaxQ) {
        err = "order/quadrature out of range";
        return false;
    }
    t.p = p; t.d = p + 1; t.q = q;
    gauss_lobatto(p, t.nodes);
    gauss_legendre(q, t.qpts, t.qwts);
    t.B.assign((size_t)q * t.d, 0.0);
    t.G.assign((size_t)q * t.d, 0.0);
    for (int a = 0; a < q; ++a) lagrange_bary(t.nodes, t.qpts[a], &t.B[(size_t)a * t.d], &t.G[(size_t)a * t.d]);
    return true;
}

bool make_l2_tables(int pu, int q, Tables1D &t, std::string &err)
{
    if (pu < 0 || pu + 1 > kMaxD || q < 1 || q > kMaxQ) {
        err = "velocity order/quadrature out of range";
        return false;
    }
    t.p = pu; t.d = pu + 1; t.q = q;
    std::vector<double> w;
    gauss_legendre(t.d, t.nodes, w);  // velocity nodes: the pu+1 Gauss-Legendre points
    gauss_legendre(q, t.qpts, t.qwts);
    t.B.assign((size_t)q * t.d, 0.0);
    t.G.assign((size_t)q * t.d, 0.0);
    for (int a = 0; a < q; ++a) lagrange_bary(t.nodes, t.qpts[a], &t.B[(size_t)a * t.d], &t.G[(size_t)a * t.d]);
    return true;
}

}  // namespace hexpa
