"""Input generators (meshes, vectors, coefficient fields); no FE arithmetic here."""
import numpy as np

STREAM_MESH = 0
STREAM_X = 1
STREAM_FIELD = 2
STREAM_AUX = 3


def _rng(seed, stream):
    return np.random.default_rng([int(seed), int(stream)])


def _lattice_vertices(n):
    """Vertex lattice of an n^3 box: index v = I + (n+1) J + (n+1)^2 K."""
    m = n + 1
    t = np.arange(m, dtype=np.float64) / n
    K, J, I = np.meshgrid(t, t, t, indexing="ij")
    return np.stack([I.ravel(), J.ravel(), K.ravel()], axis=1)


def _hex_connectivity(n):
    """Element e = ex + n ey + n^2 ez; corner c = a + 2b + 4c' at vertex (ex+a, ey+b, ez+c')."""
    m = n + 1
    ez, ey, ex = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    ex, ey, ez = ex.ravel(), ey.ravel(), ez.ravel()
    hexes = np.empty((n ** 3, 8), dtype=np.int32)
    for c in range(8):
        a, b, cc = c & 1, (c >> 1) & 1, (c >> 2) & 1
        hexes[:, c] = (ex + a) + m * (ey + b) + m * m * (ez + cc)
    return hexes


def box_mesh(n, perturb=0.1, seed=0):
    """Unit-cube mesh of n^3 hexahedra with trilinear geometry.

    Interior vertices are moved by independent U[-perturb*h, perturb*h] offsets
    in each coordinate (h = 1/n); boundary vertices stay on the exact cube.
    Returns dict(n, vert[(n+1)^3,3] float64, hex[n^3,8] int32).
    """
    n = int(n)
    vert = _lattice_vertices(n)
    if perturb:
        m = n + 1
        idx = np.arange(m ** 3)
        I, J, K = idx % m, (idx // m) % m, idx // (m * m)
        interior = (I > 0) & (I < n) & (J > 0) & (J < n) & (K > 0) & (K < n)
        h = 1.0 / n
        off = _rng(seed, STREAM_MESH).uniform(-perturb * h, perturb * h, size=vert.shape)
        vert = vert + off * interior[:, None]
    return {"n": n, "vert": np.ascontiguousarray(vert), "hex": _hex_connectivity(n)}


def affine_box_mesh(n, L, t=(0.0, 0.0, 0.0)):
    """n^3 lattice mapped by the global affine map x = L xi + t (L 3x3, det L > 0)."""
    vert = _lattice_vertices(int(n)) @ np.asarray(L, dtype=np.float64).T + np.asarray(t, dtype=np.float64)
    return {"n": int(n), "vert": np.ascontiguousarray(vert), "hex": _hex_connectivity(int(n))}


def rand_x(ndof, seed=0):
    """x ~ U[-1, 1]^ndof."""
    return _rng(seed, STREAM_X).uniform(-1.0, 1.0, size=int(ndof))


def grf_grid(seed, ell=0.1, nfft=128, period=2.0, stream=STREAM_FIELD):
    """Zero-mean, unit-variance Gaussian random field with covariance exp(-r^2/(2 ell^2)).

    Synthesised by FFT filtering of white noise on an nfft^3 periodic grid over
    [0, period)^3; the sub-grid covering [0,1]^3 (nfft/period + 1 points per
    direction, x fastest) is returned after normalising it to mean 0, std 1.
    """
    rng = _rng(seed, stream)
    w = rng.standard_normal((nfft, nfft, nfft))
    k = 2.0 * np.pi * np.fft.fftfreq(nfft, d=period / nfft)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    amp = np.exp(-0.25 * ell * ell * (kx * kx + ky * ky + kz * kz))  # sqrt of SE spectrum
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * amp))
    m = int(round(nfft / period)) + 1
    g = g[:m, :m, :m]
    g = (g - g.mean()) / g.std()
    return np.ascontiguousarray(g)  # [iz][iy][ix]


def lognormal_kappa_grid(seed, sigma=1.0, ell=0.1, nfft=128):
    """kappa = exp(sigma g) on the [0,1]^3 grid of grf_grid; returns (grid, contrast)."""
    kap = np.exp(sigma * grf_grid(seed, ell=ell, nfft=nfft))
    return np.ascontiguousarray(kap), float(kap.max() / kap.min())


def sine_kappa(xyz, amp=0.5, freq=2.0):
    """kappa(x) = 1 + amp sin(freq pi x) sin(freq pi y) sin(freq pi z)."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    w = freq * np.pi
    return 1.0 + amp * np.sin(w * x) * np.sin(w * y) * np.sin(w * z)


def u_manufactured(xyz):
    """u(x) = sin(pi x) sin(pi y) sin(pi z)."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)


def f_manufactured(xyz, amp=0.5):
    """f = -div(kappa grad u) for u = sin sin sin and kappa = 1 + amp S(x)S(y)S(z),
    S = sin(2 pi .), C = cos(2 pi .), s = sin(pi .), c = cos(pi .)."""
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    pi = np.pi
    s = [np.sin(pi * v) for v in (x, y, z)]
    c = [np.cos(pi * v) for v in (x, y, z)]
    S = [np.sin(2 * pi * v) for v in (x, y, z)]
    C = [np.cos(2 * pi * v) for v in (x, y, z)]
    kap = 1.0 + amp * S[0] * S[1] * S[2]
    u = s[0] * s[1] * s[2]
    # grad kappa . grad u
    gk_gu = amp * 2 * pi * pi * (C[0] * S[1] * S[2] * c[0] * s[1] * s[2]
                                 + S[0] * C[1] * S[2] * s[0] * c[1] * s[2]
                                 + S[0] * S[1] * C[2] * s[0] * s[1] * c[2])
    return 3 * pi * pi * kap * u - gk_gu


def trilinear_sample(grid, xyz):
    """Sample a [gz][gy][gx] grid covering [0,1]^3 at points xyz (N,3) by trilinear interpolation."""
    gz, gy, gx = grid.shape
    out = np.zeros(xyz.shape[0])
    pos = []
    for d, g in zip(range(3), (gx, gy, gz)):
        t = np.clip(xyz[:, d], 0.0, 1.0) * (g - 1)
        i0 = np.minimum(np.floor(t).astype(np.int64), g - 2)
        pos.append((i0, t - i0))
    (ix, fx), (iy, fy), (iz, fz) = pos
    for c in range(8):
        a, b, cc = c & 1, (c >> 1) & 1, (c >> 2) & 1
        wgt = (fx if a else 1 - fx) * (fy if b else 1 - fy) * (fz if cc else 1 - fz)
        out += wgt * grid[iz + cc, iy + b, ix + a]
    return out


def net_params(cin=2, ch=16, seed=0):
    """Random parameters of the 3-layer convolutional network (cin -> ch -> ch -> 1,
    3x3x3 kernels): He-normal weights rounded to FP32, small random biases.  Layout
    [W1 [ch][cin][3][3][3], b1 [ch], W2 [ch][ch][3][3][3], b2 [ch], W3 [1][ch][3][3][3], b3 [1]]."""
    rng = _rng(seed, STREAM_AUX + 4)
    W1 = rng.standard_normal((ch, cin, 3, 3, 3)) * np.sqrt(2.0 / (27 * cin))
    W2 = rng.standard_normal((ch, ch, 3, 3, 3)) * np.sqrt(2.0 / (27 * ch))
    W3 = rng.standard_normal((1, ch, 3, 3, 3)) * np.sqrt(1.0 / (27 * ch))
    b1, b2, b3 = (0.1 * rng.standard_normal(k) for k in (ch, ch, 1))
    ps = [W1, b1, W2, b2, W3, b3]
    return [p.astype(np.float32).astype(np.float64) for p in ps]


def flat_params(ps):
    """The parameter list above as one flat FP32 vector (the library's layout)."""
    return np.concatenate([np.asarray(p, dtype=np.float32).ravel() for p in ps])


def train_solution(xyz, seed, ell=0.2, nfft=64):
    """Known solution of a training system: sin(pi x) sin(pi y) sin(pi z) (1 + 0.5 g(x)),
    g a unit-variance Gaussian random field (correlation length ell) drawn from
    stream 3 with the given seed and sampled trilinearly at the points xyz [n][3]."""
    g = grf_grid(seed, ell=ell, nfft=nfft, stream=STREAM_AUX)
    return u_manufactured(xyz) * (1.0 + 0.5 * trilinear_sample(g, xyz))
