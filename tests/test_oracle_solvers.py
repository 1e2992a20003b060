"""Pins of the oracle solvers (no GPU)."""
import numpy as np
import pytest

import oracle
from oracle import solvers
import synth


def _poisson(n, p, perturb=0.1, seed=0, coeff=None):
    m = synth.box_mesh(n, perturb=perturb, seed=seed)
    P = oracle.Problem(m, p, p + 2, coeff=coeff or oracle.Coeff.sine(), ops=oracle.DIFFUSION)
    ess = oracle.box_boundary(n, p).astype(bool)
    A = oracle.Assembled(P)
    Ac = solvers.constrained(A.apply, ess)
    fq = synth.f_manufactured(P.qpoints().reshape(-1, 3)).reshape(P.nelem, -1)
    b = np.where(ess, 0.0, P.load(fq))
    dinv = 1.0 / solvers.constrained_diag(P.diag(), ess)
    return P, A, Ac, b, dinv, ess


def test_pcg_reaches_true_residual():
    P, A, Ac, b, dinv, ess = _poisson(4, 2)
    x, it, rec, true, hist = solvers.pcg(Ac, b, lambda r: dinv * r, rtol=1e-8)
    assert rec <= 1e-8 and true <= 1e-8 * 1.5
    assert np.all(x[ess] == 0.0)
    # CG (no preconditioner) converges to the same solution
    x2, it2, _, true2, _ = solvers.pcg(Ac, b, None, rtol=1e-10)
    assert true2 <= 1.5e-10
    assert np.linalg.norm(x - x2) <= 1e-6 * np.linalg.norm(x2)


def test_fcg_with_fixed_spd_preconditioner_equals_pcg():
    """With a fixed SPD preconditioner, (z_{k+1}, r_k) = 0 in exact arithmetic, so the
    Polak-Ribiere beta of FCG(1) equals the Fletcher-Reeves beta of PCG."""
    P, A, Ac, b, dinv, ess = _poisson(3, 2)
    M = lambda r: dinv * r
    xa, ia, _, _, ha = solvers.pcg(Ac, b, M, rtol=1e-9)
    xb, ib, _, _, hb = solvers.fcg(Ac, b, M, rtol=1e-9)
    assert ia == ib
    k = min(len(ha), len(hb), 15)
    np.testing.assert_allclose(ha[:k], hb[:k], rtol=1e-6)
    assert np.linalg.norm(xa - xb) <= 1e-8 * np.linalg.norm(xa)


def test_iterative_refinement_with_inexact_inner_solve():
    P, A, Ac, b, dinv, ess = _poisson(3, 2)
    inner = lambda r: solvers.pcg(Ac, r, lambda s: dinv * s, rtol=1e-2)[0]
    x, outer, hist = solvers.iterative_refinement(Ac, b, inner, rtol=1e-10)
    assert hist[-1] <= 1e-10
    assert all(hist[i + 1] < hist[i] for i in range(len(hist) - 1))


@pytest.mark.parametrize("p", [1, 2, 4])
def test_discretisation_error_rate(p):
    """Nodal error of the discrete solution of -div(kappa grad u) = f against the exact
    u = sin(pi x) sin(pi y) sin(pi z) decays like h^(p+1): the observed rate of each mesh
    halving n = 4 -> 8 -> 16 is at least p + 1 - 0.3 (a wrong sign or a dropped term in the
    operator, the load vector or the solver leaves an O(1) error that does not decay)."""
    errs = []
    for n in (4, 8, 16):
        P, A, Ac, b, dinv, ess = _poisson(n, p, perturb=0.0)
        x, *_ = solvers.pcg(Ac, b, lambda r: dinv * r, rtol=1e-13)
        errs.append(np.abs(x - synth.u_manufactured(P.nodes())).max())
        del A
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > p + 1 - 0.3), (errs, rates)
