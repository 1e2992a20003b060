"""Oracle of the learned preconditioner's network — TEST INFRASTRUCTURE ONLY.

Per element, a 3-layer convolutional network on the (p+1)^3 nodal tile:
    a1 = relu(conv(x0; W1, b1)),  a2 = relu(conv(a1; W2, b2)),  out = conv(a2; W3, b3)
with conv = 3x3x3 cross-correlation with zero padding 1 ("same" size) plus a bias,
written from the definition; the backward pass is the chain rule written out as plain
loops over the 27 taps.  Tiles are indexed [element][channel][k][j][i] (i fastest), the
same local node order as the operator (node I = i + d j + d^2 k).

The preconditioner built on it maps a residual r to
    z = W G^T ( s_e * (net(x+) - net(x-)) / 2 ),   x+- = [+-G_e r / s_e, log kappa_E]
(network part) with s_e the RMS of r over the nodes of element e and W = 1 / (element
multiplicity of each DOF), i.e. the element outputs are averaged where elements share
DOFs.  The odd part in r makes the map odd and positively homogeneous, z(a r) = a z(r)
for every real a, as a CG-type method needs of its preconditioner; the ReLU network
with biases alone is not odd.
"""
import numpy as np


def conv3d(x, W, b):
    """x [E][Cin][n][n][n], W [Cout][Cin][3][3][3], b [Cout] -> [E][Cout][n][n][n]."""
    E, Cin, n = x.shape[0], x.shape[1], x.shape[2]
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    out = np.broadcast_to(b[None, :, None, None, None], (E, W.shape[0], n, n, n)).copy()
    for tz in range(3):
        for ty in range(3):
            for tx in range(3):
                patch = xp[:, :, tz:tz + n, ty:ty + n, tx:tx + n]
                out += np.einsum("oc,eckji->eokji", W[:, :, tz, ty, tx], patch)
    return out


def conv3d_backward(x, W, dout):
    """Gradients of sum(dout * conv3d(x, W, b)) w.r.t. x, W and b."""
    E, Cin, n = x.shape[0], x.shape[1], x.shape[2]
    xp = np.pad(x, ((0, 0), (0, 0), (1, 1), (1, 1), (1, 1)))
    dxp = np.zeros_like(xp)
    dW = np.zeros_like(W)
    for tz in range(3):
        for ty in range(3):
            for tx in range(3):
                patch = xp[:, :, tz:tz + n, ty:ty + n, tx:tx + n]
                dW[:, :, tz, ty, tx] = np.einsum("eokji,eckji->oc", dout, patch)
                dxp[:, :, tz:tz + n, ty:ty + n, tx:tx + n] += np.einsum("oc,eokji->eckji", W[:, :, tz, ty, tx], dout)
    db = dout.sum(axis=(0, 2, 3, 4))
    return dxp[:, :, 1:-1, 1:-1, 1:-1], dW, db


def relu(z):
    return np.maximum(z, 0.0)


class Net:
    """Three conv layers: cin -> ch -> ch -> 1, ReLU between."""

    def __init__(self, params):
        self.W1, self.b1, self.W2, self.b2, self.W3, self.b3 = [np.asarray(p, dtype=np.float64) for p in params]

    def params(self):
        return [self.W1, self.b1, self.W2, self.b2, self.W3, self.b3]

    def forward(self, x0):
        z1 = conv3d(x0, self.W1, self.b1)
        a1 = relu(z1)
        z2 = conv3d(a1, self.W2, self.b2)
        a2 = relu(z2)
        out = conv3d(a2, self.W3, self.b3)
        self.cache = (x0, z1, a1, z2, a2)
        return out

    def backward(self, dout):
        x0, z1, a1, z2, a2 = self.cache
        da2, dW3, db3 = conv3d_backward(a2, self.W3, dout)
        dz2 = da2 * (z2 > 0)
        da1, dW2, db2 = conv3d_backward(a1, self.W2, dz2)
        dz1 = da1 * (z1 > 0)
        dx0, dW1, db1 = conv3d_backward(x0, self.W1, dz1)
        return [dW1, db1, dW2, db2, dW3, db3], dx0


def element_tiles(v, elem_dofs, d):
    """G_e v for every element as [E][d][d][d] ([k][j][i])."""
    return v[elem_dofs].reshape(-1, d, d, d)


def multiplicity(elem_dofs, ndof):
    return np.bincount(elem_dofs.ravel(), minlength=ndof).astype(np.float64)


def net_input(r, logk_tiles, elem_dofs, d):
    """Channels [+-r_E / s_e, log kappa_E] for both signs, stacked as [2E][2][d][d][d]
    (the first E tiles with +r); s_e = RMS of r over the element's nodes (1 if zero)."""
    rt = element_tiles(r, elem_dofs, d)
    s = np.sqrt((rt ** 2).reshape(rt.shape[0], -1).mean(axis=1))
    s = np.where(s > 0.0, s, 1.0)
    lk = logk_tiles.reshape(-1, d, d, d)
    xp = np.stack([rt / s[:, None, None, None], lk], axis=1)
    xm = np.stack([-rt / s[:, None, None, None], lk], axis=1)
    return np.concatenate([xp, xm], axis=0), s


def precond_nn(net, r, logk_tiles, elem_dofs, d, ndof, ess=None):
    """Network part of the preconditioner: z = W G^T (s_e (out(x+) - out(x-)) / 2)."""
    x0, s = net_input(r, logk_tiles, elem_dofs, d)
    o = net.forward(x0)[:, 0]
    E = s.size
    out = 0.5 * (o[:E] - o[E:]) * s[:, None, None, None]
    z = np.zeros(ndof)
    np.add.at(z, elem_dofs.ravel(), out.reshape(-1))
    z /= multiplicity(elem_dofs, ndof)
    if ess is not None:
        z[ess] = 0.0
    return z, (x0, s)


def loss_and_grads(net, r, t, logk_tiles, elem_dofs, d, ndof, ess, Amul=None):
    """Loss of the network part z of the preconditioner against the target t and its
    gradient w.r.t. the parameters:
        Amul None:  L = ||z - t||^2 / ||t||^2                 (free DOFs)
        Amul given: L = (z - t)^T A (z - t) / t^T A t          (A = Amul, symmetric)
    with dL/dz = 2 (z - t) / ||t||^2, resp. 2 A (z - t) / t^T A t, pulled back through the
    averaging W, the scaling by s_e and the network."""
    z, (x0, s) = precond_nn(net, r, logk_tiles, elem_dofs, d, ndof, ess)
    free = ~ess
    diff = np.where(free, z - t, 0.0)
    tf = np.where(free, t, 0.0)
    if Amul is None:
        Ad, At = diff, tf
    else:
        Ad, At = Amul(diff), Amul(tf)
    den = float(tf @ At)
    L = float(diff @ Ad) / den
    gz = np.where(free, 2.0 * Ad / den, 0.0)          # dL/dz
    gz = gz / multiplicity(elem_dofs, ndof)           # through the averaging W
    gout = element_tiles(gz, elem_dofs, d) * s[:, None, None, None]  # through s_e * out
    gout = 0.5 * np.concatenate([gout, -gout], axis=0)                # through the odd part
    grads, _ = net.backward(gout[:, None])
    return L, grads


def adam_step(params, grads, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """Adam (Kingma & Ba): one update of every parameter array, t = 1, 2, ..."""
    out = []
    for i, (p, g) in enumerate(zip(params, grads)):
        m[i] = b1 * m[i] + (1 - b1) * g
        v[i] = b2 * v[i] + (1 - b2) * g * g
        mh = m[i] / (1 - b1 ** t)
        vh = v[i] / (1 - b2 ** t)
        out.append(p - lr * mh / (np.sqrt(vh) + eps))
    return out
