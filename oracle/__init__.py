"""CPU FP64 oracle — TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It shares no code with the HIP library
(``paper_2603_09038_amd``): the operator arithmetic lives in ``oracle.c`` (plain
quadrature loops, dense element matrices) and the solvers in ``solvers.py``.
Inputs come from the ``synth`` fixtures.
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

MASS = 1
DIFFUSION = 2
COEFF_CONST, COEFF_SINE, COEFF_GRID = 0, 1, 2


class _Coeff(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("value", ctypes.c_double), ("amp", ctypes.c_double),
                ("freq", ctypes.c_double), ("grid", ctypes.c_void_p), ("gx", ctypes.c_int32),
                ("gy", ctypes.c_int32), ("gz", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(quiet=True)
        _lib = ctypes.CDLL(LIB)
        _lib.orc_num_threads.restype = ctypes.c_int
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


class Coeff:
    """Coefficient kappa(x): constant, value + amp sin(freq pi x)sin(..y)sin(..z), or a
    [gz][gy][gx] grid over [0,1]^3 sampled by trilinear interpolation."""

    def __init__(self, kind=COEFF_CONST, value=1.0, amp=0.0, freq=0.0, grid=None):
        self.grid = None if grid is None else _f64(grid)
        gz, gy, gx = (0, 0, 0) if grid is None else self.grid.shape
        self.c = _Coeff(kind, value, amp, freq, None if grid is None else self.grid.ctypes.data, gx, gy, gz)

    def at(self, xyz):
        """kappa at physical points xyz [n][3]."""
        xyz = _f64(xyz).reshape(-1, 3)
        out = np.zeros(xyz.shape[0])
        lib().orc_coeff_points(ctypes.byref(self.c), ctypes.c_int64(xyz.shape[0]), _p(xyz), _p(out))
        return out

    @staticmethod
    def const(v=1.0):
        return Coeff(COEFF_CONST, value=v)

    @staticmethod
    def sine(value=1.0, amp=0.5, freq=2.0):
        return Coeff(COEFF_SINE, value=value, amp=amp, freq=freq)

    @staticmethod
    def from_grid(grid):
        return Coeff(COEFF_GRID, grid=grid)


def num_threads():
    return lib().orc_num_threads()


# ---------------------------------------------------------------- 1-D tables
def gauss(q):
    x, w = np.zeros(q), np.zeros(q)
    if lib().orc_gauss(ctypes.c_int(q), _p(x), _p(w)):
        raise RuntimeError("orc_gauss failed")
    return x, w


def gll(p):
    x = np.zeros(p + 1)
    if lib().orc_gll(ctypes.c_int(p), _p(x)):
        raise RuntimeError("orc_gll failed")
    return x


def lagrange(nodes, t):
    nodes = _f64(nodes)
    n = nodes.size
    l, dl = np.zeros(n), np.zeros(n)
    lib().orc_lagrange(ctypes.c_int(n), _p(nodes), ctypes.c_double(t), _p(l), _p(dl))
    return l, dl


# ---------------------------------------------------------------------- maps
def box_elem_dofs(n, p):
    d = p + 1
    out = np.zeros((n ** 3, d ** 3), dtype=np.int32)
    lib().orc_box_elem_dofs(ctypes.c_int(n), ctypes.c_int(p), _p(out))
    return out


def box_boundary(n, p):
    M = n * p + 1
    out = np.zeros(M ** 3, dtype=np.uint8)
    lib().orc_box_boundary(ctypes.c_int(n), ctypes.c_int(p), _p(out))
    return out


def box_ndof(n, p):
    return (n * p + 1) ** 3


# ------------------------------------------------------------------ operator
class Problem:
    """A mesh (synth.box_mesh dict), order p, q-point Gauss rule, coefficient and ops mask."""

    def __init__(self, mesh, p, q, coeff=None, ops=DIFFUSION, elem_dofs=None):
        self.mesh, self.p, self.q, self.ops = mesh, int(p), int(q), int(ops)
        self.coeff = coeff if coeff is not None else Coeff.const(1.0)
        self.vert = _f64(mesh["vert"])
        self.hex = _i32(mesh["hex"])
        self.nelem = self.hex.shape[0]
        self.d = self.p + 1
        self.nd = self.d ** 3
        if elem_dofs is None:
            elem_dofs = box_elem_dofs(mesh["n"], self.p)
        self.elem_dofs = _i32(elem_dofs)
        self.ndof = int(self.elem_dofs.max()) + 1

    # dense element matrices of a subset (or all)
    def elem_matrices(self, subset=None):
        sub = None if subset is None else _i32(subset)
        ns = self.nelem if sub is None else sub.size
        Ae = np.zeros((ns, self.nd, self.nd))
        md = np.zeros(1)
        rc = lib().orc_elem_matrices(ctypes.c_int64(ns), None if sub is None else _p(sub), _p(self.vert),
                                     _p(self.hex), ctypes.c_int(self.p), ctypes.c_int(self.q),
                                     ctypes.byref(self.coeff.c), ctypes.c_int(self.ops), _p(Ae), _p(md))
        if rc:
            raise RuntimeError("orc_elem_matrices failed")
        self.min_detj = float(md[0])
        return Ae

    def apply(self, x, subset=None):
        x = _f64(x)
        y = np.zeros(self.ndof)
        sub = None if subset is None else _i32(subset)
        rc = lib().orc_apply(ctypes.c_int64(self.nelem), ctypes.c_int64(0 if sub is None else sub.size),
                             None if sub is None else _p(sub), _p(self.vert), _p(self.hex), _p(self.elem_dofs),
                             ctypes.c_int(self.p), ctypes.c_int(self.q), ctypes.byref(self.coeff.c),
                             ctypes.c_int(self.ops), ctypes.c_int64(self.ndof), _p(x), _p(y))
        if rc:
            raise RuntimeError("orc_apply failed")
        return y

    def diag(self):
        dg = np.zeros(self.ndof)
        rc = lib().orc_diag(ctypes.c_int64(self.nelem), _p(self.vert), _p(self.hex), _p(self.elem_dofs),
                            ctypes.c_int(self.p), ctypes.c_int(self.q), ctypes.byref(self.coeff.c),
                            ctypes.c_int(self.ops), ctypes.c_int64(self.ndof), _p(dg))
        if rc:
            raise RuntimeError("orc_diag failed")
        return dg

    def apply_rows(self, x, rows):
        """y[rows] computed from the element rows only (for checks at full size)."""
        rows = np.asarray(rows, dtype=np.int64)
        ed = self.elem_dofs
        hit = np.isin(ed, rows)
        pe, pl = np.nonzero(hit)
        pos = {int(r): i for i, r in enumerate(rows)}
        po = np.array([pos[int(v)] for v in ed[pe, pl]], dtype=np.int32)
        out = np.zeros(rows.size)
        pe, pl = _i32(pe), _i32(pl)
        rc = lib().orc_apply_rows(ctypes.c_int64(pe.size), _p(pe), _p(pl), _p(po), ctypes.c_int64(rows.size),
                                  _p(self.vert), _p(self.hex), _p(ed), ctypes.c_int(self.p), ctypes.c_int(self.q),
                                  ctypes.byref(self.coeff.c), ctypes.c_int(self.ops), _p(_f64(x)), _p(out))
        if rc:
            raise RuntimeError("orc_apply_rows failed")
        return out

    def qpoints(self):
        q = self.q
        out = np.zeros((self.nelem, q ** 3, 3))
        if lib().orc_qpoints(ctypes.c_int64(self.nelem), _p(self.vert), _p(self.hex), ctypes.c_int(q), _p(out)):
            raise RuntimeError("orc_qpoints failed")
        return out

    def nodes(self):
        out = np.zeros((self.ndof, 3))
        if lib().orc_nodes(ctypes.c_int64(self.nelem), _p(self.vert), _p(self.hex), _p(self.elem_dofs),
                           ctypes.c_int(self.p), _p(out)):
            raise RuntimeError("orc_nodes failed")
        return out

    def load(self, fq):
        fq = _f64(fq).reshape(self.nelem, self.q ** 3)
        b = np.zeros(self.ndof)
        if lib().orc_load(ctypes.c_int64(self.nelem), _p(self.vert), _p(self.hex), _p(self.elem_dofs),
                          ctypes.c_int(self.p), ctypes.c_int(self.q), _p(fq), ctypes.c_int64(self.ndof), _p(b)):
            raise RuntimeError("orc_load failed")
        return b


class Assembled:
    """Element matrices stored once; y = sum_e G_e^T A_e G_e x (for solver tests)."""

    def __init__(self, prob):
        self.prob = prob
        self.Ae = prob.elem_matrices()
        self.ndof = prob.ndof

    def apply(self, x):
        y = np.zeros(self.ndof)
        lib().orc_apply_assembled(ctypes.c_int64(self.prob.nelem), ctypes.c_int(self.prob.nd), _p(self.Ae),
                                  _p(self.prob.elem_dofs), ctypes.c_int64(self.ndof), _p(_f64(x)), _p(y))
        return y


class MixedProblem:
    """The off-diagonal blocks of the acoustic block operator (the paper's eq. (4)) on a
    mesh: pressure in the continuous order-p space (GLL nodes), velocity in the
    discontinuous order-pu space (Lagrange on pu+1 Gauss-Legendre points per axis, three
    scalar components, element-local vectors [nelem][3][(pu+1)^3]), q-point Gauss rule.
    G p = (grad p, tau) and -G^T u = -(u, grad v); lumped masses by row sums."""

    def __init__(self, mesh, p=4, pu=3, q=5, rho=1.0, bulk=1.0):
        self.mesh, self.p, self.pu, self.q = mesh, int(p), int(pu), int(q)
        self.rho, self.bulk = float(rho), float(bulk)
        self.vert = _f64(mesh["vert"])
        self.hex = _i32(mesh["hex"])
        self.nelem = self.hex.shape[0]
        self.nd = (self.p + 1) ** 3
        self.nu = (self.pu + 1) ** 3
        self.elem_dofs = _i32(box_elem_dofs(mesh["n"], self.p))
        self.ndof = int(self.elem_dofs.max()) + 1
        self.nvel = self.nelem * 3 * self.nu

    def elem_matrices(self, subset=None):
        sub = None if subset is None else _i32(subset)
        ns = self.nelem if sub is None else sub.size
        Ge = np.zeros((ns, 3 * self.nu, self.nd))
        if lib().orc_mixed_elem_matrices(ctypes.c_int64(ns), None if sub is None else _p(sub), _p(self.vert),
                                         _p(self.hex), ctypes.c_int(self.p), ctypes.c_int(self.pu),
                                         ctypes.c_int(self.q), _p(Ge)):
            raise RuntimeError("orc_mixed_elem_matrices failed")
        return Ge

    def apply(self, u, pv):
        """(yu, yp) = (G p, -G^T u)."""
        u, pv = _f64(u).ravel(), _f64(pv)
        yu = np.zeros(self.nvel)
        yp = np.zeros(self.ndof)
        if lib().orc_mixed_apply(ctypes.c_int64(self.nelem), _p(self.vert), _p(self.hex), _p(self.elem_dofs),
                                 ctypes.c_int(self.p), ctypes.c_int(self.pu), ctypes.c_int(self.q),
                                 ctypes.c_int64(self.ndof), _p(u), _p(pv), _p(yu), _p(yp)):
            raise RuntimeError("orc_mixed_apply failed")
        return yu, yp

    def lumped(self):
        """(mu [nelem][nu], mp [ndof]): velocity mass rows (one per node, the same for each
        component) and the assembled pressure mass rows."""
        mu = np.zeros(self.nelem * self.nu)
        mp = np.zeros(self.ndof)
        if lib().orc_mixed_lumped(ctypes.c_int64(self.nelem), _p(self.vert), _p(self.hex), _p(self.elem_dofs),
                                  ctypes.c_int(self.p), ctypes.c_int(self.pu), ctypes.c_int(self.q),
                                  ctypes.c_double(self.rho), ctypes.c_double(self.bulk), ctypes.c_int64(self.ndof),
                                  _p(mu), _p(mp)):
            raise RuntimeError("orc_mixed_lumped failed")
        return mu, mp

    def velocity_mass_rows(self):
        """mu expanded to the velocity layout [nelem][3][nu]."""
        mu, _ = self.lumped()
        return np.repeat(mu.reshape(self.nelem, 1, self.nu), 3, axis=1).ravel()

    def rhs(self, u, pv, mu3=None, mp=None):
        """Time derivative of the semi-discrete system M [u; p]' = -A [u; p] with the
        off-diagonal blocks of eq. (4) (no boundary terms: u . n = 0 on the box):
        u' = -Mu^{-1} G p, p' = Mp^{-1} G^T u."""
        if mu3 is None:
            mu3 = self.velocity_mass_rows()
        if mp is None:
            _, mp = self.lumped()
        yu, yp = self.apply(u, pv)
        return -yu / mu3, -yp / mp

    def rk4(self, u, pv, dt, nsteps):
        from .solvers import rk4
        mu3 = self.velocity_mass_rows()
        _, mp = self.lumped()
        return rk4(lambda a, b: self.rhs(a, b, mu3, mp), _f64(u).ravel().copy(), _f64(pv).copy(), dt, nsteps)
