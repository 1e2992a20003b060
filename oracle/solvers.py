"""Oracle solvers in numpy — TEST INFRASTRUCTURE ONLY.

Written from the textbook definitions:
  * preconditioned CG: Saad, Iterative Methods for Sparse Linear Systems, Alg. 9.1;
  * flexible CG, FCG(1): Notay (2000) / Golub & Ye (1999), Polak-Ribiere beta;
  * iterative refinement: r = b - A x in FP64, correction by an inner solve, x += d.
The stop test everywhere is ||r_k||_2 <= rtol ||b||_2 on the recursively updated
residual, with the true residual reported on exit.
"""
import numpy as np


def constrained(apply_fn, ess):
    """A_c = (I - P) A (I - P) + P with P the indicator of the essential DOFs."""
    ess = np.asarray(ess, dtype=bool)

    def op(x):
        xi = np.where(ess, 0.0, x)
        y = apply_fn(xi)
        return np.where(ess, x, y)

    return op


def constrained_diag(diag, ess):
    return np.where(np.asarray(ess, dtype=bool), 1.0, diag)


def pcg(A, b, Minv=None, rtol=1e-8, max_it=10000, x0=None):
    """Preconditioned CG; returns (x, iters, rel_res_recursive, rel_res_true, history)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A(x)
    nb = np.linalg.norm(b)
    z = r if Minv is None else Minv(r)
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while it < max_it and hist[-1] > rtol:
        Ap = A(p)
        alpha = rz / (p @ Ap)
        x += alpha * p
        r -= alpha * Ap
        it += 1
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            break
        z = r if Minv is None else Minv(r)
        rz_new = r @ z
        beta = rz_new / rz
        rz = rz_new
        p = z + beta * p
    true = np.linalg.norm(b - A(x)) / nb
    return x, it, hist[-1], true, hist


def fcg(A, b, Minv, rtol=1e-8, max_it=10000, x0=None):
    """Flexible CG with one-term truncation (FCG(1)):
    beta_k = (z_{k+1}, r_{k+1} - r_k) / (z_k, r_k)."""
    x = np.zeros_like(b) if x0 is None else np.array(x0, dtype=np.float64)
    r = b - A(x)
    nb = np.linalg.norm(b)
    z = Minv(r)
    p = z.copy()
    rz = r @ z
    hist = [np.linalg.norm(r) / nb]
    it = 0
    while it < max_it and hist[-1] > rtol:
        Ap = A(p)
        alpha = rz / (p @ Ap)
        x += alpha * p
        r_old = r.copy()
        r = r - alpha * Ap
        it += 1
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            break
        z = Minv(r)
        beta = (z @ (r - r_old)) / rz
        rz = r @ z
        p = z + beta * p
    true = np.linalg.norm(b - A(x)) / nb
    return x, it, hist[-1], true, hist


def iterative_refinement(A64, b, inner_solve, rtol=1e-8, max_outer=100):
    """x_{k+1} = x_k + d_k with d_k ~ A^{-1} r_k from inner_solve(r_k), r_k = b - A64 x_k in FP64."""
    x = np.zeros_like(b)
    nb = np.linalg.norm(b)
    hist = []
    for _ in range(max_outer):
        r = b - A64(x)
        hist.append(np.linalg.norm(r) / nb)
        if hist[-1] <= rtol:
            break
        x = x + inner_solve(r)
    return x, len(hist) - 1, hist


def rk4(f, u, p, dt, nsteps):
    """Classical fourth-order Runge-Kutta for the pair (u, p) with (u', p') = f(u, p):
    k1 = f(x), k2 = f(x + dt/2 k1), k3 = f(x + dt/2 k2), k4 = f(x + dt k3),
    x <- x + dt/6 (k1 + 2 k2 + 2 k3 + k4)."""
    u, p = np.array(u, dtype=np.float64), np.array(p, dtype=np.float64)
    for _ in range(int(nsteps)):
        k1u, k1p = f(u, p)
        k2u, k2p = f(u + 0.5 * dt * k1u, p + 0.5 * dt * k1p)
        k3u, k3p = f(u + 0.5 * dt * k2u, p + 0.5 * dt * k2p)
        k4u, k4p = f(u + dt * k3u, p + dt * k3p)
        u = u + dt / 6.0 * (k1u + 2.0 * k2u + 2.0 * k3u + k4u)
        p = p + dt / 6.0 * (k1p + 2.0 * k2p + 2.0 * k3p + k4p)
    return u, p
