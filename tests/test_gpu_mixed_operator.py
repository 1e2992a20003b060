"""The paper's own operator on MI355X: the fused kernel of the off-diagonal blocks of the
acoustic operator (eq. (4)), the lumped masses and the RK4 stepper, against the CPU
oracle (dense element matrices by quadrature loops).

Bars: the fused apply and the masses reach the element-matrix results up to rounding
order (sum factorization, atomic scatter): 1e-12 normwise in the 2-norm and the max-norm,
as for the H1 operators.  RK4 states after a few steps: 1e-11 (four applies per step,
each within 1e-12, composed linearly with O(1) amplification over a few steps)."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def hx():
    import torch  # noqa: F401
    from paper_2603_09038_amd import hexpa
    return hexpa


def _t(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return max(np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("p,pu,q,n", [(4, 3, 5, 3), (2, 1, 3, 8)])
def test_fused_apply_matches_the_oracle(hx, p, pu, q, n):
    """yu = G p and yp = -G^T u against the dense element matrices, with the persistent
    grid uncapped (one group per workgroup) and capped (8 and 3 workgroups: each walks
    several element groups)."""
    mesh = synth.box_mesh(n, perturb=0.1, seed=60 + p)
    m = hx.MixedOperator(mesh, p, pu, q)
    P = oracle.MixedProblem(mesh, p, pu, q)
    assert (m.ndof_p, m.ndof_u) == (P.ndof, P.nvel)
    rng = np.random.default_rng(61)
    u = rng.uniform(-1, 1, P.nvel)
    pv = rng.uniform(-1, 1, P.ndof)
    ru, rp = P.apply(u, pv)
    ud, pd = _t(u), _t(pv)
    ngroups = -(-P.nelem // m.info["elems_per_block"])
    for cap in (0, 8, 3):
        m.set_grid_cap(cap)
        yu, yp = m.apply(ud, pd)
        assert _rel(yu.cpu().numpy(), ru) <= TOL, (cap, _rel(yu.cpu().numpy(), ru))
        assert _rel(yp.cpu().numpy(), rp) <= TOL, (cap, _rel(yp.cpu().numpy(), rp))
    assert ngroups >= 2 * 3
    m.close()


def test_lumped_masses_match_the_oracle(hx):
    mesh = synth.box_mesh(3, perturb=0.1, seed=62)
    m = hx.MixedOperator(mesh, rho=1.5, bulk=2.5)
    P = oracle.MixedProblem(mesh, rho=1.5, bulk=2.5)
    mu, mp = m.lumped()
    ru, rp = P.lumped()
    assert _rel(mu.cpu().numpy(), ru) <= TOL and _rel(mp.cpu().numpy(), rp) <= TOL
    m.close()


def test_rk4_matches_the_oracle(hx):
    mesh = synth.box_mesh(2, perturb=0.1, seed=63)
    m = hx.MixedOperator(mesh)
    P = oracle.MixedProblem(mesh)
    xp = oracle.Problem(mesh, 4, 5).nodes()
    p0 = np.exp(-20 * ((xp - 0.45) ** 2).sum(1))
    u0 = np.random.default_rng(64).uniform(-0.1, 0.1, P.nvel)
    ud, pd = _t(u0), _t(p0)
    m.rk4(ud, pd, 2e-3, 6)
    ur, pr = P.rk4(u0, p0, 2e-3, 6)
    assert _rel(ud.cpu().numpy(), ur) <= 1e-11 and _rel(pd.cpu().numpy(), pr) <= 1e-11
    m.close()


def test_full_size_properties(hx):
    """48^3 perturbed mesh (the benchmark's 28.4 M DOFs): sampled elements against their
    oracle element matrices; a linear pressure gives yu = a_c times the oracle's lumped
    velocity mass rows; a constant velocity has no divergence at interior pressure nodes;
    and the two blocks are adjoint, u . (G p) = -p . (-G^T u)."""
    import torch
    n = 48
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    m = hx.MixedOperator(mesh)
    P = oracle.MixedProblem(mesh)
    rng = np.random.default_rng(65)
    u = rng.uniform(-1, 1, P.nvel)
    pv = rng.uniform(-1, 1, P.ndof)
    yu, yp = m.apply(_t(u), _t(pv))
    yu = yu.cpu().numpy()
    sub = np.unique(np.concatenate([rng.integers(0, P.nelem, 200), [0, P.nelem - 1]])).astype(np.int32)
    Ge = P.elem_matrices(sub)
    ref = np.einsum("sri,si->sr", Ge, pv[P.elem_dofs[sub]])
    got = yu.reshape(P.nelem, -1)[sub]
    assert _rel(got, ref) <= TOL
    # adjointness over the whole vectors
    lhs = float(np.dot(u, yu))
    rhs = float(np.dot(pv, yp.cpu().numpy()))
    assert abs(lhs + rhs) <= 1e-12 * np.abs(u).sum() * np.abs(yu).max()
    # linear pressure
    xp = oracle.Problem(mesh, 4, 5).nodes()
    a = np.array([0.4, -0.9, 0.25])
    yu_lin, _ = m.apply(torch.zeros(P.nvel, dtype=torch.float64, device="cuda"), _t(xp @ a - 0.3))
    mu, _ = P.lumped()
    expect = (a[None, :, None] * mu.reshape(P.nelem, 1, P.nu)).ravel()
    assert _rel(yu_lin.cpu().numpy(), expect) <= TOL
    # constant velocity
    uc = np.zeros((P.nelem, 3, P.nu))
    uc[:, 0], uc[:, 1], uc[:, 2] = 0.7, 0.1, -0.5
    _, ypc = m.apply(_t(uc), torch.zeros(P.ndof, dtype=torch.float64, device="cuda"))
    ypc = ypc.cpu().numpy()
    interior = ~oracle.box_boundary(n, 4).astype(bool)
    assert np.abs(ypc[interior]).max() <= TOL * np.abs(ypc).max()
    m.close()
