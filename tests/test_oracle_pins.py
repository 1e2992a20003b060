"""Pins of the CPU oracle against facts the mathematics fixes (no GPU).

Each test ties one oracle function to something other than itself: closed forms,
exactness of Gauss quadrature, polynomial reproduction, patch tests, an
independent lattice construction, and brute-force evaluation with numpy's own
quadrature and polynomial routines.  A dropped term, a wrong sign or index, or a
transposed Jacobian in the oracle fails at least one of them.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


# ------------------------------------------------------------------ 1-D
def test_gll_closed_forms():
    assert np.allclose(oracle.gll(1), [0.0, 1.0], atol=0, rtol=0)
    np.testing.assert_allclose(oracle.gll(2), [0.0, 0.5, 1.0], atol=1e-15)
    s = 1 / np.sqrt(5)
    np.testing.assert_allclose(oracle.gll(3), [0.0, (1 - s) / 2, (1 + s) / 2, 1.0], atol=1e-15)
    s = np.sqrt(3 / 7)
    np.testing.assert_allclose(oracle.gll(4), [0.0, (1 - s) / 2, 0.5, (1 + s) / 2, 1.0], atol=1e-15)


@pytest.mark.parametrize("p", [2, 3, 4, 5, 6, 7, 8])
def test_gll_roots_and_lobatto_exactness(p):
    """GLL nodes at every order the library instantiates, pinned two ways that share nothing
    with the oracle's bisection: (i) the interior nodes are the roots of P_p' as numpy's
    Legendre class finds them (companion-matrix eigenvalues); (ii) the interpolatory rule
    on the nodes (weights = integrals of the Lagrange basis on the nodes) is
    exact for x^k, k <= 2p - 1, the property that singles out the Lobatto points among
    (p+1)-point rules through both endpoints, and at degree 2p its error is the Lobatto
    remainder -n (n-1)^3 2^(2n-1) ((n-2)!)^4 / ((2n-1) ((2n-2)!)^3) f^(2n-2) on [-1,1]
    (n = p + 1 points), mapped to [0,1]."""
    from math import factorial
    x = oracle.gll(p)
    t = np.sort(np.polynomial.legendre.Legendre.basis(p).deriv().roots().real)
    np.testing.assert_allclose(x[1:-1], (t + 1) / 2, atol=1e-13)
    # w_i = integral of l_i: the product formula at numpy's Gauss points (exact for degree p)
    tg, wg = np.polynomial.legendre.leggauss(p + 1)
    tg, wg = (tg + 1) / 2, wg / 2
    w = np.array([wg @ np.prod([(tg - x[j]) / (x[i] - x[j]) for j in range(p + 1) if j != i], axis=0)
                  for i in range(p + 1)])
    for k in range(2 * p):
        assert abs(w @ x ** k - 1 / (k + 1)) < 1e-13, (p, k)
    n = p + 1
    e11 = -n * (n - 1) ** 3 * 2.0 ** (2 * n - 1) * factorial(n - 2) ** 4 / ((2 * n - 1) * factorial(2 * n - 2) ** 3)
    rem = 0.5 * e11 * factorial(2 * p) / 2.0 ** (2 * p)  # f = x^(2p) on [0,1]
    err = 1 / (2 * p + 1) - w @ x ** (2 * p)
    assert abs(err - rem) <= 1e-6 * abs(rem), (p, err, rem)


def test_gauss_closed_forms():
    x, w = oracle.gauss(2)
    s = 1 / np.sqrt(3)
    np.testing.assert_allclose(x, [(1 - s) / 2, (1 + s) / 2], atol=1e-15)
    np.testing.assert_allclose(w, [0.5, 0.5], atol=1e-15)
    x, w = oracle.gauss(3)
    s = np.sqrt(3 / 5)
    np.testing.assert_allclose(x, [(1 - s) / 2, 0.5, (1 + s) / 2], atol=1e-15)
    np.testing.assert_allclose(w, [5 / 18, 8 / 18, 5 / 18], atol=1e-15)


@pytest.mark.parametrize("q", [1, 2, 3, 4, 6, 8, 10, 12, 14])
def test_gauss_exactness(q):
    x, w = oracle.gauss(q)
    assert abs(w.sum() - 1) < 1e-14
    for k in range(2 * q):
        assert abs(w @ x ** k - 1 / (k + 1)) < 1e-14, (q, k)
    # degree 2q: the error equals the Gauss remainder (q!)^4 / ((2q+1) ((2q)!)^2) on [0,1]
    from math import factorial
    rem = factorial(q) ** 4 / ((2 * q + 1) * factorial(2 * q) ** 2)
    err = 1 / (2 * q + 1) - w @ x ** (2 * q)
    assert abs(err - rem) <= 1e-6 * rem + 1e-15
    # agrees with numpy's Golub-Welsch rule mapped to [0,1]
    t, wt = np.polynomial.legendre.leggauss(q)
    np.testing.assert_allclose(x, (t + 1) / 2, atol=2e-15)
    np.testing.assert_allclose(w, wt / 2, atol=2e-15)


@pytest.mark.parametrize("p", [1, 2, 3, 4, 6, 8])
def test_lagrange_properties(p):
    nodes = oracle.gll(p)
    for j, t in enumerate(nodes):
        l, dl = oracle.lagrange(nodes, t)
        np.testing.assert_allclose(l, np.eye(p + 1)[j], atol=1e-13)
    for t in np.linspace(-0.1, 1.1, 13):
        l, dl = oracle.lagrange(nodes, t)
        assert abs(l.sum() - 1) < 1e-12
        assert abs(dl.sum()) < 1e-10
        for m in range(p + 1):  # reproduction of t^m and its derivative
            assert abs(l @ nodes ** m - t ** m) < 1e-11
            assert abs(dl @ nodes ** m - (m * t ** (m - 1) if m else 0.0)) < 1e-9
    # derivative against numpy's polynomial built from the roots
    for i in range(p + 1):
        others = np.delete(nodes, i)
        poly = np.polynomial.Polynomial.fromroots(others)
        poly = poly / poly(nodes[i])
        for t in (0.13, 0.5, 0.91):
            l, dl = oracle.lagrange(nodes, t)
            assert abs(dl[i] - poly.deriv()(t)) < 1e-10


# ------------------------------------------------------------------ maps
@pytest.mark.parametrize("n,p", [(1, 1), (2, 2), (3, 4), (2, 5)])
def test_box_map_against_coordinate_hash(n, p):
    """Independent construction: number the distinct node positions of an unperturbed
    box in (z, y, x) lexicographic order and look every element node up by position."""
    ed = oracle.box_elem_dofs(n, p)
    d = p + 1
    g = oracle.gll(p)
    keys = []
    for ez, ey, ex in itertools.product(range(n), repeat=3):
        for k, j, i in itertools.product(range(d), repeat=3):
            # integer lattice position avoids floating ties
            keys.append(((ez * p + k), (ey * p + j), (ex * p + i)))
    uniq = sorted(set(keys))
    pos = {key: r for r, key in enumerate(uniq)}
    ref = np.array([pos[kk] for kk in keys], dtype=np.int32).reshape(n ** 3, d ** 3)
    assert np.array_equal(ed, ref)
    assert len(uniq) == oracle.box_ndof(n, p)
    # and the positions behind those integers are the GLL lattice
    assert g[0] == 0.0 and g[-1] == 1.0
    M = n * p + 1
    mk = oracle.box_boundary(n, p).reshape(M, M, M)
    assert mk[1:-1, 1:-1, 1:-1].sum() == 0 and mk.sum() == M ** 3 - max(M - 2, 0) ** 3


def test_nodes_match_affine_lattice():
    n, p = 3, 3
    m = synth.box_mesh(n, perturb=0.0)
    P = oracle.Problem(m, p, p + 2)
    X = P.nodes()
    M = n * p + 1
    g = oracle.gll(p)
    lat = np.concatenate([(e + g[:-1]) / n for e in range(n)] + [[1.0]])
    K, J, I = np.meshgrid(lat, lat, lat, indexing="ij")
    np.testing.assert_allclose(X, np.stack([I.ravel(), J.ravel(), K.ravel()], 1), atol=1e-15)
    assert X.shape[0] == M ** 3


# --------------------------------------------------------------- geometry
def test_qpoints_and_volume():
    m = synth.box_mesh(3, perturb=0.0)
    P = oracle.Problem(m, 2, 3, ops=oracle.MASS)
    xq = P.qpoints()
    x, _ = oracle.gauss(3)
    # element 0 occupies [0,1/3]^3: qp (a,b,c) at (x_a, x_b, x_c)/3, a fastest
    ref = np.array([[x[a], x[b], x[c]] for c in range(3) for b in range(3) for a in range(3)]) / 3
    np.testing.assert_allclose(xq[0], ref, atol=1e-16)
    # the load vector of f = 1 sums to the volume, on a perturbed mesh too
    m = synth.box_mesh(4, perturb=0.1, seed=3)
    P = oracle.Problem(m, 3, 5, ops=oracle.MASS)
    b = P.load(np.ones((P.nelem, 125)))
    assert abs(b.sum() - 1.0) < 1e-14


# ------------------------------------------------------------------ mass
@pytest.mark.parametrize("p", [1, 2, 3, 4])
def test_mass_volume_and_linear_moments(p):
    m = synth.box_mesh(3, perturb=0.1, seed=1)
    P = oracle.Problem(m, p, p + 2, ops=oracle.MASS)
    one = np.ones(P.ndof)
    assert abs(one @ P.apply(one) - 1.0) < 1e-14
    X = P.nodes()  # physical coordinates are in the space (trilinear geometry, p >= 1)
    Mx = P.apply(X[:, 0])
    assert abs(one @ Mx - 0.5) < 1e-14            # int x
    assert abs(X[:, 0] @ Mx - 1 / 3) < 1e-14      # int x^2
    assert abs(X[:, 1] @ Mx - 1 / 4) < 1e-14      # int x y
    assert abs(X[:, 2] @ P.apply(X[:, 1]) - 1 / 4) < 1e-14


def _fd_jacobian(Xc, xi):
    """Exact Jacobian of a trilinear map by differences along each (linear) direction."""
    def xmap(s):
        out = np.zeros(3)
        for c in range(8):
            bits = (c & 1, (c >> 1) & 1, (c >> 2) & 1)
            out += Xc[c] * np.prod([s[k] if bits[k] else 1 - s[k] for k in range(3)])
        return out
    J = np.zeros((3, 3))
    for s in range(3):
        hi, lo = list(xi), list(xi)
        hi[s], lo[s] = 1.0, 0.0
        J[:, s] = xmap(hi) - xmap(lo)
    return xmap(xi), J


def _brute_element(p, Xc, nq, diffusion):
    """Element matrix with numpy's Gauss rule, numpy polynomials and difference Jacobians."""
    nodes = oracle.gll(p)
    d = p + 1
    polys = []
    for i in range(d):
        pl = np.polynomial.Polynomial.fromroots(np.delete(nodes, i))
        polys.append(pl / pl(nodes[i]))
    t, wt = np.polynomial.legendre.leggauss(nq)
    t, wt = (t + 1) / 2, wt / 2
    L = np.array([[pl(s) for pl in polys] for s in t])
    dL = np.array([[pl.deriv()(s) for pl in polys] for s in t])
    A = np.zeros((d ** 3, d ** 3))
    for a, b, c in itertools.product(range(nq), repeat=3):
        _, J = _fd_jacobian(Xc, (t[a], t[b], t[c]))
        det = np.linalg.det(J)
        w = wt[a] * wt[b] * wt[c] * det
        phi = np.einsum("k,j,i->kji", L[c], L[b], L[a]).ravel()
        if not diffusion:
            A += w * np.outer(phi, phi)
        else:
            gref = np.stack([np.einsum("k,j,i->kji", L[c], L[b], dL[a]).ravel(),
                             np.einsum("k,j,i->kji", L[c], dL[b], L[a]).ravel(),
                             np.einsum("k,j,i->kji", dL[c], L[b], L[a]).ravel()], 1)
            g = np.linalg.solve(J.T, gref.T).T
            A += w * g @ g.T
    return A


@pytest.mark.parametrize("p", [1, 2, 3])
def test_one_element_mass_brute_force(p):
    """Mass integrand on a trilinear element is a polynomial of degree <= 2p+2 per axis:
    both the oracle (q = p+2) and the brute force (numpy, q = p+6) are exact."""
    m = synth.box_mesh(1)
    rng = np.random.default_rng(7)
    Xc = m["vert"][m["hex"][0]] + rng.uniform(-0.12, 0.12, (8, 3))
    mesh = {"n": 1, "vert": Xc, "hex": np.arange(8, dtype=np.int32)[None]}
    P = oracle.Problem(mesh, p, p + 2, ops=oracle.MASS)
    A = P.elem_matrices()[0]
    B = _brute_element(p, Xc, p + 6, diffusion=False)
    assert np.abs(A - B).max() <= 1e-14 * np.abs(B).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_one_element_diffusion_brute_force(p):
    """Diffusion integrand is rational on non-affine elements: compare at the same
    (high) quadrature order against independent code; then check convergence of the
    oracle's own rule toward it."""
    m = synth.box_mesh(1)
    rng = np.random.default_rng(11)
    Xc = m["vert"][m["hex"][0]] + rng.uniform(-0.12, 0.12, (8, 3))
    mesh = {"n": 1, "vert": Xc, "hex": np.arange(8, dtype=np.int32)[None]}
    nq = p + 8
    A = oracle.Problem(mesh, p, nq, ops=oracle.DIFFUSION).elem_matrices()[0]
    B = _brute_element(p, Xc, nq, diffusion=True)
    assert np.abs(A - B).max() <= 1e-13 * np.abs(B).max()
    A2 = oracle.Problem(mesh, p, p + 2, ops=oracle.DIFFUSION).elem_matrices()[0]
    assert np.abs(A2 - B).max() <= 5e-2 * np.abs(B).max()


# --------------------------------------------------------------- diffusion
@pytest.mark.parametrize("p", [1, 2, 4])
def test_diffusion_constants_and_patch_test(p):
    m = synth.box_mesh(3, perturb=0.1, seed=2)
    P = oracle.Problem(m, p, p + 2, ops=oracle.DIFFUSION)
    one = np.ones(P.ndof)
    K1 = P.apply(one)
    assert np.abs(K1).max() < 1e-13
    X = P.nodes()
    g = np.array([0.3, -1.1, 0.7])
    u = X @ g + 0.25
    Ku = P.apply(u)
    interior = oracle.box_boundary(3, p) == 0
    # interior rows of K applied to a physical linear function vanish (exact quadrature)
    assert np.abs(Ku[interior]).max() < 1e-13
    # energy of a linear function = |g|^2 * volume
    assert abs(u @ Ku - g @ g) < 1e-13
    h = np.array([-0.5, 0.2, 0.9])
    assert abs((X @ h) @ Ku - g @ h) < 1e-13


def _mono_int(a, b):
    """int_0^1 x^a x^b dx"""
    return 1.0 / (a + b + 1)


def _mono_grad_int(e1, e2):
    """int over the unit cube of grad(x^a y^b z^c) . grad(x^d y^e z^f)."""
    tot = 0.0
    for ax in range(3):
        t = 1.0
        for k in range(3):
            a, b = e1[k], e2[k]
            if k == ax:
                if a == 0 or b == 0:
                    t = 0.0
                    break
                t *= a * b / (a + b - 1)
            else:
                t *= _mono_int(a, b)
        tot += t
    return tot


@pytest.mark.parametrize("p", [2, 3])
def test_diffusion_monomials_unperturbed(p):
    n = 2
    m = synth.box_mesh(n, perturb=0.0)
    P = oracle.Problem(m, p, p + 1, ops=oracle.DIFFUSION)
    X = P.nodes()
    rng = np.random.default_rng(0)
    exps = [tuple(rng.integers(0, p + 1, 3)) for _ in range(5)] + [(p, p, p), (1, 0, 0)]
    for e1 in exps:
        u = np.prod(X ** np.array(e1), axis=1)
        Ku = P.apply(u)
        for e2 in exps:
            v = np.prod(X ** np.array(e2), axis=1)
            assert abs(v @ Ku - _mono_grad_int(e1, e2)) < 1e-12, (e1, e2)


def test_diffusion_sheared_affine():
    """Total degree <= p polynomials on x = L xi + t: v^T K u = int grad u . grad v
    evaluated by change of variables with numpy's Gauss rule (exact for polynomials)."""
    p, n = 3, 2
    L = np.array([[1.0, 0.3, 0.1], [0.0, 0.8, -0.2], [0.1, 0.0, 1.2]])
    tvec = np.array([0.2, -0.1, 0.5])
    m = synth.affine_box_mesh(n, L, tvec)
    P = oracle.Problem(m, p, p + 2, ops=oracle.DIFFUSION)
    X = P.nodes()
    polys = [((1, 0, 0),), ((0, 1, 1),), ((1, 1, 1),), ((2, 0, 1),), ((0, 3, 0),)]
    Linv = np.linalg.inv(L)
    t, wt = np.polynomial.legendre.leggauss(8)
    t, wt = (t + 1) / 2, wt / 2
    pts = np.array(list(itertools.product(t, t, t)))
    wts = np.prod(np.array(list(itertools.product(wt, wt, wt))), axis=1) * np.linalg.det(L)
    xs = pts @ L.T + tvec

    def grad_mono(e, x):
        g = np.zeros_like(x)
        for k in range(3):
            if e[k]:
                ee = list(e)
                ee[k] -= 1
                g[:, k] = e[k] * np.prod(x ** np.array(ee), axis=1)
        return g

    for (e1,) in polys:
        u = np.prod(X ** np.array(e1), axis=1)
        Ku = P.apply(u)
        for (e2,) in polys:
            v = np.prod(X ** np.array(e2), axis=1)
            exact = np.sum(wts * np.sum(grad_mono(e1, xs) * grad_mono(e2, xs), axis=1))
            assert abs(v @ Ku - exact) < 1e-11 * max(1.0, abs(exact)), (e1, e2)
    del Linv


@pytest.mark.parametrize("p", [2, 5])
def test_mass_plus_diffusion_is_the_sum(p):
    """ops = MASS | DIFFUSION assembles both terms in one pass over the quadrature points;
    it must equal the mass result plus the diffusion result (a dropped or doubled term in
    the combined path fails), element matrices and global apply alike, on a perturbed mesh
    with a variable coefficient."""
    m = synth.box_mesh(2, perturb=0.1, seed=6)
    c = oracle.Coeff.sine()
    Pm = oracle.Problem(m, p, p + 2, coeff=c, ops=oracle.MASS)
    Pk = oracle.Problem(m, p, p + 2, coeff=c, ops=oracle.DIFFUSION)
    Pb = oracle.Problem(m, p, p + 2, coeff=c, ops=oracle.MASS | oracle.DIFFUSION)
    Am, Ak, Ab = Pm.elem_matrices(), Pk.elem_matrices(), Pb.elem_matrices()
    assert np.abs(Ab - (Am + Ak)).max() <= 1e-14 * np.abs(Ab).max()
    # both parts are present with their own size: neither is negligible against the other
    assert np.abs(Am).max() > 1e-3 * np.abs(Ak).max()
    x = synth.rand_x(Pb.ndof, 3)
    yb, ym, yk = Pb.apply(x), Pm.apply(x), Pk.apply(x)
    assert np.linalg.norm(yb - ym - yk) <= 1e-14 * np.linalg.norm(yb)
    np.testing.assert_allclose(Pb.diag(), Pm.diag() + Pk.diag(), rtol=1e-14, atol=0)


@pytest.mark.parametrize("ops", [oracle.MASS, oracle.DIFFUSION, oracle.MASS | oracle.DIFFUSION])
def test_symmetry_definiteness(ops):
    m = synth.box_mesh(2, perturb=0.1, seed=5)
    P = oracle.Problem(m, 2, 4, coeff=oracle.Coeff.sine(), ops=ops)
    Ae = P.elem_matrices()
    for A in Ae:
        assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
        ev = np.linalg.eigvalsh(A)
        if ops & oracle.MASS:
            assert ev.min() > 0
        else:
            assert ev.min() > -1e-13 * ev.max()
            assert np.sum(ev < 1e-10 * ev.max()) == 1  # only constants in the kernel
    # global apply equals the assembled apply, and diag equals the element diagonals
    A = oracle.Assembled(P)
    x = synth.rand_x(P.ndof, 0)
    np.testing.assert_allclose(A.apply(x), P.apply(x), atol=1e-13)
    dg = np.zeros(P.ndof)
    np.add.at(dg, P.elem_dofs.ravel(), np.einsum("eii->ei", Ae).ravel())
    np.testing.assert_allclose(P.diag(), dg, atol=1e-14)
    rows = [0, 7, 13, P.ndof - 1]
    np.testing.assert_allclose(P.apply_rows(x, rows), A.apply(x)[rows], atol=1e-13)


def test_coefficients_enter_linearly():
    m = synth.box_mesh(2, perturb=0.1, seed=5)
    x = synth.rand_x(oracle.box_ndof(2, 2), 1)
    ya = oracle.Problem(m, 2, 4, coeff=oracle.Coeff.const(2.5), ops=3).apply(x)
    yb = oracle.Problem(m, 2, 4, coeff=oracle.Coeff.const(1.0), ops=3).apply(x)
    np.testing.assert_allclose(ya, 2.5 * yb, rtol=1e-13, atol=1e-14)
    # a grid coefficient holding a constant reproduces the constant
    grid = np.full((5, 6, 7), 2.5)
    yc = oracle.Problem(m, 2, 4, coeff=oracle.Coeff.from_grid(grid), ops=3).apply(x)
    np.testing.assert_allclose(yc, ya, rtol=1e-13, atol=1e-14)
    # a grid holding the linear function 1 + x is interpolated exactly
    gx = np.linspace(0, 1, 7)
    grid = np.broadcast_to(1.0 + gx[None, None, :], (5, 6, 7)).copy()
    M1 = oracle.Problem(m, 2, 4, coeff=oracle.Coeff.from_grid(grid), ops=oracle.MASS)
    one = np.ones(M1.ndof)
    assert abs(one @ M1.apply(one) - 1.5) < 1e-14  # int (1 + x) over the cube
