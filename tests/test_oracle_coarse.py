"""Pins of the oracle's coarse level (no GPU): the p = 1 -> p interpolation reproduces
functions that are trilinear in every cell and is a partition of unity; the fixed-
iteration coarse solve becomes the exact constrained inverse once the iteration count
reaches the number of free coarse DOFs (CG terminates in exact arithmetic)."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from oracle.coarse import CoarseLevel, prolongation
import synth


@pytest.mark.parametrize("n,p", [(2, 2), (3, 4), (2, 3)])
def test_prolongation_reproduces_cellwise_trilinear_functions(n, p):
    P = prolongation(n, p)
    M, C = n * p + 1, n + 1
    x = oracle.gll(p)
    # lattice coordinate of fine index I: element ex = min(I // p, n - 1) plus its GLL node
    fine = np.array([min(I // p, n - 1) + x[I - min(I // p, n - 1) * p] for I in range(M)])
    f = lambda X, Y, Z: 1.0 + 2.0 * X - Y + 0.5 * X * Y * Z - 0.25 * Y * Z
    cz, cy, cx = np.meshgrid(np.arange(C), np.arange(C), np.arange(C), indexing="ij")
    fz, fy, fx = np.meshgrid(fine, fine, fine, indexing="ij")
    u1 = f(cx, cy, cz).ravel()
    np.testing.assert_allclose(P @ u1, f(fx, fy, fz).ravel(), rtol=0, atol=1e-13)
    np.testing.assert_allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0, atol=1e-14)
    # coarse vertices coincide with fine nodes: those rows are unit rows
    for a in range(C):
        I = a * p
        row = P.getrow(I + M * (0 + M * 0)).toarray().ravel()
        assert row[a] == pytest.approx(1.0) and np.count_nonzero(np.abs(row) > 1e-15) == 1


def test_coarse_solve_with_enough_iterations_is_the_exact_inverse():
    n, p = 3, 2
    mesh = synth.box_mesh(n, perturb=0.1, seed=1)
    grid, _ = synth.lognormal_kappa_grid(2, sigma=1.0, ell=0.2, nfft=16)
    cl = CoarseLevel(mesh, n, p, oracle.Coeff.from_grid(grid))
    free = ~cl.ess1
    nf = int(free.sum())
    # assembled constrained coarse matrix from unit vectors
    N1 = cl.prob.ndof
    A = np.column_stack([cl.A1c(np.eye(N1)[:, j]) for j in range(N1)])
    r1 = np.where(free, synth.rand_x(N1, 3), 0.0)
    u = cl.solve(r1, nf + 5)
    np.testing.assert_allclose(u, np.linalg.solve(A, r1), rtol=1e-9, atol=1e-12)
    # fewer iterations: an approximation whose A-norm error decreases monotonically
    errs = []
    exact = np.linalg.solve(A, r1)
    for k in (1, 2, 4):
        e = cl.solve(r1, k) - exact
        errs.append(e @ A @ e)
    assert errs[0] > errs[1] > errs[2]
