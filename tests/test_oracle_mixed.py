"""Pins of the oracle for the mixed H1 x L2 blocks of the acoustic operator (the paper's
eq. (4)) and its RK4 driver (Sec. II-C), checked against mathematics that does not go
through the oracle: exact integrals of polynomials, the divergence theorem, the volume of
the cube, and the matrix exponential of the semi-discrete system."""
import numpy as np
import pytest
from numpy.polynomial import legendre as npleg

import oracle
import synth


def _gl01(m):
    t, _ = npleg.leggauss(m)
    return (t + 1.0) / 2.0


def _gll01(p):
    inner = npleg.Legendre.basis(p).deriv().roots()
    return np.concatenate([[0.0], (np.sort(inner.real) + 1.0) / 2.0, [1.0]])


def _h1_lattice(n, p):
    """Physical coordinates of the pressure DOFs on the unperturbed n^3 box."""
    xi = _gll01(p)
    M = n * p + 1
    idx = np.arange(M)
    c1 = (idx // p) / n + xi[idx % p] / n
    c1[-1] = 1.0
    K, J, I = np.meshgrid(c1, c1, c1, indexing="ij")
    return np.stack([I.ravel(), J.ravel(), K.ravel()], 1)


def _l2_nodes(n, pu):
    """Physical coordinates of the velocity nodes [nelem][nu][3] on the unperturbed box."""
    du = pu + 1
    t = _gl01(du)
    out = np.zeros((n ** 3, du ** 3, 3))
    for e in range(n ** 3):
        ex, ey, ez = e % n, (e // n) % n, e // (n * n)
        for J in range(du ** 3):
            j1, j2, j3 = J % du, (J // du) % du, J // (du * du)
            out[e, J] = [(ex + t[j1]) / n, (ey + t[j2]) / n, (ez + t[j3]) / n]
    return out


@pytest.mark.parametrize("p,pu,q", [(4, 3, 5), (2, 1, 3)])
def test_monomials_integrate_exactly(p, pu, q):
    """u^T G p = integral of grad p . tau for p = x^a y^b z^c (degree <= p per axis) and
    tau = x^d y^e z^f e_m (degree <= pu per axis) on the unit cube: the integrand has
    degree <= p + pu - 1 per axis, which q-point Gauss integrates exactly."""
    n = 2
    mesh = synth.box_mesh(n, perturb=0.0)
    P = oracle.MixedProblem(mesh, p, pu, q)
    xp = _h1_lattice(n, p)
    xu = _l2_nodes(n, pu)
    rng = np.random.default_rng(p)
    for _ in range(12):
        a, b, c = rng.integers(0, p + 1, 3)
        d, e, f = rng.integers(0, pu + 1, 3)
        m = int(rng.integers(0, 3))
        pv = xp[:, 0] ** a * xp[:, 1] ** b * xp[:, 2] ** c
        tau = np.zeros((P.nelem, 3, P.nu))
        tau[:, m, :] = xu[..., 0] ** d * xu[..., 1] ** e * xu[..., 2] ** f
        yu, yp = P.apply(tau.ravel(), pv)
        ex = [a, b, c]
        ey = [d, e, f]
        if ex[m] == 0:
            exact = 0.0
        else:
            exact = ex[m] / (ex[m] + ey[m])
            for s in range(3):
                if s != m:
                    exact /= ex[s] + ey[s] + 1
        assert abs(tau.ravel() @ yu - exact) <= 1e-13 * max(1.0, abs(exact)), (a, b, c, d, e, f, m)
        # and through the transposed block: -p^T (G^T tau) is the same number
        assert abs(-(pv @ yp) - exact) <= 1e-13 * max(1.0, abs(exact))


def test_linear_pressure_gives_the_velocity_mass_rows():
    """For p = a . x + b (exactly in the pressure space on a trilinear mesh, since x is
    trilinear in the reference coordinates), (grad p, psi_J e_c) = a_c integral psi_J,
    the lumped velocity mass row: pins G and the lumped mass against each other."""
    mesh = synth.box_mesh(3, perturb=0.1, seed=4)
    P = oracle.MixedProblem(mesh)
    xp = oracle.Problem(mesh, 4, 5).nodes()
    a = np.array([0.3, -1.1, 0.7])
    yu, _ = P.apply(np.zeros(P.nvel), xp @ a + 0.4)
    mu, _ = P.lumped()
    expect = (a[None, :, None] * mu.reshape(P.nelem, 1, P.nu)).ravel()
    np.testing.assert_allclose(yu, expect, rtol=0, atol=1e-13 * np.abs(expect).max())


def test_constant_velocity_has_no_interior_divergence():
    """-(u, grad v) for constant u equals minus the boundary flux of u against v, so it
    vanishes at every pressure node off the boundary, on a perturbed mesh too."""
    n, p = 3, 4
    mesh = synth.box_mesh(n, perturb=0.1, seed=5)
    P = oracle.MixedProblem(mesh)
    u = np.zeros((P.nelem, 3, P.nu))
    u[:, 0], u[:, 1], u[:, 2] = 0.6, -0.2, 1.3
    _, yp = P.apply(u.ravel(), np.zeros(P.ndof))
    interior = ~oracle.box_boundary(n, p).astype(bool)
    assert np.abs(yp[interior]).max() <= 1e-14 * np.abs(yp).max()
    assert np.abs(yp[~interior]).max() > 1e-3


def test_lumped_masses_sum_to_the_volume():
    mesh = synth.box_mesh(3, perturb=0.1, seed=6)
    P = oracle.MixedProblem(mesh, rho=2.0, bulk=4.0)
    mu, mp = P.lumped()
    assert abs(mu.sum() - 2.0) <= 1e-13 and abs(mp.sum() - 0.25) <= 1e-13
    assert mu.min() > 0 and mp.min() > 0


def test_rk4_is_fourth_order_against_the_matrix_exponential():
    """The semi-discrete system x' = L x (u' = -Mu^{-1} G p, p' = Mp^{-1} G^T u) is linear:
    x(T) = expm(T L) x(0).  RK4's global error falls by 2^4 when the step halves."""
    from scipy.linalg import expm
    mesh = synth.box_mesh(1, perturb=0.0)
    mesh["vert"] = mesh["vert"] + np.random.default_rng(7).uniform(-0.05, 0.05, mesh["vert"].shape)
    P = oracle.MixedProblem(mesh, p=2, pu=1, q=3)
    nv, npr = P.nvel, P.ndof
    N = nv + npr
    L = np.zeros((N, N))
    for j in range(N):
        x = np.zeros(N)
        x[j] = 1.0
        du, dp = P.rhs(x[:nv], x[nv:])
        L[:, j] = np.concatenate([du, dp])
    rng = np.random.default_rng(8)
    x0 = rng.standard_normal(N)
    T = 0.05
    xT = expm(T * L) @ x0
    errs = []
    for steps in (8, 16, 32):
        u, pv = P.rk4(x0[:nv], x0[nv:], T / steps, steps)
        errs.append(np.linalg.norm(np.concatenate([u, pv]) - xT))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 19.0 and 13.0 < r2 < 19.0, errs


def test_rk4_energy_is_nearly_conserved():
    """E = (u^T Mu u + p^T Mp p) / 2 is an invariant of the semi-discrete system (the
    blocks are skew-adjoint in the mass inner product); RK4 dissipates it by O(dt^4)."""
    mesh = synth.box_mesh(2, perturb=0.1, seed=9)
    P = oracle.MixedProblem(mesh)
    mu3 = P.velocity_mass_rows()
    _, mp = P.lumped()
    xp = oracle.Problem(mesh, 4, 5).nodes()
    p0 = np.exp(-20 * ((xp - 0.5) ** 2).sum(1))
    u0 = np.zeros(P.nvel)
    E = lambda u, p: 0.5 * (mu3 @ (u * u) + mp @ (p * p))  # noqa: E731
    u, pv = P.rk4(u0, p0, 2e-3, 20)
    e0, e1 = E(u0, p0), E(u, pv)
    assert e1 <= e0 and (e0 - e1) / e0 < 1e-6, (e0, e1)
    assert np.abs(u).max() > 1e-3  # the pressure pulse set the velocity in motion
