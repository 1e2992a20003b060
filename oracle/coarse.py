"""Oracle of the p = 1 coarse correction of the two-level preconditioner —
TEST INFRASTRUCTURE ONLY (imported by tests, the smoke check and the CPU baseline).

    z_c = P1 A1^{-1} P1^T r

P1 is the interpolation of a p = 1 (trilinear) finite-element function at the nodes of
the order-p space on the same mesh: in every element the p = 1 Lagrange basis on the
nodes {0, 1} per axis is evaluated at the element's GLL nodes (tensor products), and the
value at a global node is that element's interpolant there (the p = 1 function is
continuous, so every element holding the node gives the same value).  The restriction
is the transpose.  A1 is the p = 1 operator on the same mesh and coefficient with 3-point
Gauss quadrature, constrained on the box boundary; A1^{-1} is approximated by a fixed
number of Jacobi-PCG iterations from zero (Saad, Alg. 9.1).
"""
import numpy as np
import scipy.sparse as sp

import oracle
from . import solvers


def prolongation(n, p):
    """Sparse P1 [ndof_p][ndof_1] on the structured n^3 box."""
    d = p + 1
    ed_p = oracle.box_elem_dofs(n, p)
    ed_1 = oracle.box_elem_dofs(n, 1)
    x = oracle.gll(p)
    l1 = np.array([oracle.lagrange(np.array([0.0, 1.0]), t)[0] for t in x])  # [d][2]
    rows, cols, vals = [], [], []
    for e in range(n ** 3):
        for k in range(d):
            for j in range(d):
                for i in range(d):
                    g = ed_p[e, i + d * (j + d * k)]
                    for c in range(2):
                        for b in range(2):
                            for a in range(2):
                                w = l1[i, a] * l1[j, b] * l1[k, c]
                                if w != 0.0:
                                    rows.append(g)
                                    cols.append(ed_1[e, a + 2 * (b + 2 * c)])
                                    vals.append(w)
    P = sp.coo_matrix((vals, (rows, cols)), shape=(oracle.box_ndof(n, p), oracle.box_ndof(n, 1))).tocsr()
    # a node shared by elements was entered once per element with the same weights
    mult = sp.coo_matrix((np.ones(len(rows)), (rows, cols)), shape=P.shape).tocsr()
    P.data /= mult.data
    return P


class CoarseLevel:
    """The coarse operator on a box mesh and its fixed-iteration Jacobi-PCG solve."""

    def __init__(self, mesh, n, p, coeff, ops=oracle.DIFFUSION, constrained=True):
        self.P = prolongation(n, p)
        self.prob = oracle.Problem(mesh, 1, 3, coeff=coeff, ops=ops)
        self.ess1 = oracle.box_boundary(n, 1).astype(bool) if constrained else np.zeros(self.prob.ndof, bool)
        self.A1c = solvers.constrained(self.prob.apply, self.ess1)
        self.dinv1 = 1.0 / solvers.constrained_diag(self.prob.diag(), self.ess1)
        self.ess = oracle.box_boundary(n, p).astype(bool) if constrained else None

    def solve(self, r1, iters):
        r1 = np.where(self.ess1, 0.0, r1)
        u, *_ = solvers.pcg(self.A1c, r1, lambda v: self.dinv1 * v, rtol=0.0, max_it=iters)
        return u

    def correction(self, r, iters):
        z = self.P @ self.solve(self.P.T @ r, iters)
        if self.ess is not None:
            z[self.ess] = 0.0
        return z
