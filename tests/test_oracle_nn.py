"""Pins of the oracle network (no GPU): the convolution against a direct per-point sum,
the backward pass against central finite differences, and Adam against its closed form
on a quadratic."""
import numpy as np
import pytest

from oracle import nn
import oracle
import synth


def test_conv3d_matches_direct_sum():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 3, 4, 4, 4))
    W = rng.standard_normal((2, 3, 3, 3, 3))
    b = rng.standard_normal(2)
    y = nn.conv3d(x, W, b)
    for e in range(2):
        for o in range(2):
            for k in range(4):
                for j in range(4):
                    for i in range(4):
                        acc = b[o]
                        for c in range(3):
                            for tz in range(3):
                                for ty in range(3):
                                    for tx in range(3):
                                        kk, jj, ii = k + tz - 1, j + ty - 1, i + tx - 1
                                        if 0 <= kk < 4 and 0 <= jj < 4 and 0 <= ii < 4:
                                            acc += W[o, c, tz, ty, tx] * x[e, c, kk, jj, ii]
                        assert abs(y[e, o, k, j, i] - acc) < 1e-12


def test_conv3d_identity_kernel():
    x = np.random.default_rng(1).standard_normal((1, 1, 5, 5, 5))
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 1, 1, 1] = 1.0
    np.testing.assert_array_equal(nn.conv3d(x, W, np.zeros(1)), x)
    W = np.zeros((1, 1, 3, 3, 3))
    W[0, 0, 1, 1, 2] = 1.0  # reads the +x neighbour
    y = nn.conv3d(x, W, np.zeros(1))
    np.testing.assert_array_equal(y[0, 0, :, :, :-1], x[0, 0, :, :, 1:])
    assert np.all(y[0, 0, :, :, -1] == 0.0)


def _setup(p=2, n=2, seed=3):
    mesh = synth.box_mesh(n, perturb=0.1, seed=seed)
    d = p + 1
    ed = oracle.box_elem_dofs(n, p)
    ndof = oracle.box_ndof(n, p)
    ess = oracle.box_boundary(n, p).astype(bool)
    rng = np.random.default_rng(seed)
    logk = rng.standard_normal(ed.shape)
    r = np.where(ess, 0.0, rng.standard_normal(ndof))
    t = np.where(ess, 0.0, rng.standard_normal(ndof))
    return mesh, d, ed, ndof, ess, logk, r, t


def test_network_gradients_against_central_differences():
    mesh, d, ed, ndof, ess, logk, r, t = _setup()
    net = nn.Net(synth.net_params(2, 4, seed=1))
    L0, grads = nn.loss_and_grads(net, r, t, logk, ed, d, ndof, ess)
    rng = np.random.default_rng(5)
    h = 1e-6
    for pi, P in enumerate(net.params()):
        flat = P.reshape(-1)
        for idx in rng.choice(flat.size, min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            Lp, _ = nn.loss_and_grads(net, r, t, logk, ed, d, ndof, ess)
            flat[idx] = old - h
            Lm, _ = nn.loss_and_grads(net, r, t, logk, ed, d, ndof, ess)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            g = grads[pi].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (pi, idx, fd, g)


def test_preconditioner_is_odd_homogeneous_and_averages():
    mesh, d, ed, ndof, ess, logk, r, t = _setup()
    net = nn.Net(synth.net_params(2, 4, seed=2))
    z1, _ = nn.precond_nn(net, r, logk, ed, d, ndof, ess)
    z2, _ = nn.precond_nn(net, 3.5 * r, logk, ed, d, ndof, ess)
    np.testing.assert_allclose(z2, 3.5 * z1, rtol=1e-12, atol=1e-14)
    # a network whose output is the constant 1 (zero weights, bias 1) gives z = s-average
    ps = [np.zeros_like(q) for q in net.params()]
    ps[5] = np.ones(1)
    z, (x0, s) = nn.precond_nn(nn.Net(ps), r, logk, ed, d, ndof, None)
    assert np.all(z == 0.0)  # a constant output has no odd part
    # a network whose output is relu(first input channel) (identity centre taps): the odd
    # part (relu(x) - relu(-x)) / 2 = x / 2 of x = r_E / s_e, so z = W G^T r_E / 2 = r / 2
    ps = [np.zeros_like(q) for q in net.params()]
    ps[0][0, 0, 1, 1, 1] = 1.0   # a1[0] = relu(+-r/s)
    ps[2][0, 0, 1, 1, 1] = 1.0   # a2[0] = a1[0]
    ps[4][0, 0, 1, 1, 1] = 1.0   # out = a2[0]
    z, _ = nn.precond_nn(nn.Net(ps), r, logk, ed, d, ndof, None)
    np.testing.assert_allclose(z, 0.5 * r, rtol=1e-12, atol=1e-14)
    # oddness and homogeneity for negative scalings too
    z1, _ = nn.precond_nn(net, r, logk, ed, d, ndof, ess)
    z3, _ = nn.precond_nn(net, -2.5 * r, logk, ed, d, ndof, ess)
    np.testing.assert_allclose(z3, -2.5 * z1, rtol=1e-12, atol=1e-14)


def test_adam_minimises_a_quadratic():
    p = [np.array([3.0, -2.0])]
    m, v = [np.zeros(2)], [np.zeros(2)]
    for t in range(1, 3001):
        g = [2.0 * p[0]]
        p = nn.adam_step(p, g, m, v, t, lr=1e-2)
    assert np.abs(p[0]).max() < 1e-3
    # first step moves every coordinate by lr (bias-corrected m/sqrt(v) = sign(g))
    p = [np.array([3.0, -2.0])]
    m, v = [np.zeros(2)], [np.zeros(2)]
    q = nn.adam_step(p, [np.array([0.7, -1e-3])], m, v, 1, lr=0.1)
    np.testing.assert_allclose(q[0], [2.9, -1.9], rtol=0, atol=1e-6)


def test_energy_loss_gradients_against_central_differences():
    mesh, d, ed, ndof, ess, logk, r, t = _setup(p=2, n=2, seed=4)
    P = oracle.Problem(mesh, 2, 4, coeff=oracle.Coeff.sine(), ops=oracle.DIFFUSION)
    from oracle import solvers
    Ac = solvers.constrained(P.apply, ess)
    net = nn.Net(synth.net_params(2, 4, seed=3))
    L0, grads = nn.loss_and_grads(net, r, t, logk, ed, d, ndof, ess, Amul=Ac)
    assert 0.0 < L0
    rng = np.random.default_rng(6)
    h = 1e-6
    for pi, Pm in enumerate(net.params()):
        flat = Pm.reshape(-1)
        for idx in rng.choice(flat.size, min(4, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            Lp, _ = nn.loss_and_grads(net, r, t, logk, ed, d, ndof, ess, Amul=Ac)
            flat[idx] = old - h
            Lm, _ = nn.loss_and_grads(net, r, t, logk, ed, d, ndof, ess, Amul=Ac)
            flat[idx] = old
            fd = (Lp - Lm) / (2 * h)
            g = grads[pi].reshape(-1)[idx]
            assert abs(fd - g) <= 1e-6 * max(1.0, abs(fd)) + 1e-8, (pi, idx, fd, g)
    # the energy loss of t itself against 0 output is 1 (z = 0 network: all-zero parameters)
    zero = nn.Net([np.zeros_like(q) for q in net.params()])
    L1, _ = nn.loss_and_grads(zero, r, t, logk, ed, d, ndof, ess, Amul=Ac)
    assert L1 == pytest.approx(1.0, rel=1e-14)
