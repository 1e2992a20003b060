"""ctypes binding of libhexpa.so (argument marshalling only).

Every call below forwards to the C function of the same name declared in
``include/hexpa.h``; all arithmetic runs in the library's HIP kernels.  Device
vectors are torch tensors on the GPU (float64, contiguous); the library works on
the caller's current torch stream.  There is no CPU fallback: if the shared
library is missing or fails to load, importing this module raises.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhexpa.so")

PA_OK = 0
PA_ERR_ARG, PA_ERR_HIP, PA_ERR_UNSUPPORTED, PA_ERR_MESH = -1, -2, -3, -4
PA_ERR_NOT_CONVERGED, PA_ERR_BREAKDOWN, PA_ERR_IO = -5, -6, -7
PA_MASS, PA_DIFFUSION = 1, 2
PA_COEFF_CONST, PA_COEFF_SINE, PA_COEFF_GRID = 0, 1, 2
PA_VARIANT_MFMA, PA_VARIANT_VALU, PA_VARIANT_MFMA_COLORED, PA_VARIANT_MFMA_UNFUSED, PA_VARIANT_VALU_UNFUSED = 0, 1, 2, 3, 4
PA_VARIANT_MFMA_MF, PA_VARIANT_VALU_MF = 5, 6
PA_CG_PLAIN, PA_CG_JACOBI, PA_CG_MIXED_IR, PA_CG_FCG, PA_CG_MIXED_FCG, PA_CG_MIXED_RU = 0, 1, 2, 3, 4, 5
PA_LP_LOSS_ENERGY, PA_LP_LOSS_L2 = 0, 1
PA_LP_FP16, PA_LP_BF16 = 0, 1
PA_LP_CAPTURE_FCG, PA_LP_CAPTURE_JACOBI = 0, 1

# every symbol include/hexpa.h declares
EXPORTS = ("pa_setup", "pa_apply", "pa_apply_add", "pa_apply_lp", "pa_apply_unfused_noalloc", "pa_apply_constrained", "pa_diag", "pa_load", "pa_qpoints", "pa_nodes",
           "pa_get_elem_dofs", "pa_get_ess", "pa_set_variant", "pa_set_grid_cap", "pa_info", "pa_destroy", "pa_last_error",
           "cg_solve", "pa_debug_mfma_f64", "pa_debug_mfma16",
           "pa_lp_create", "pa_lp_bind", "pa_lp_configure", "pa_lp_num_params", "pa_lp_get_params",
           "pa_lp_set_params", "pa_lp_logk", "pa_lp_apply", "pa_lp_coarse", "pa_lp_net", "pa_lp_loss_grad",
           "pa_lp_train_step", "pa_lp_train", "pa_lp_save", "pa_lp_load", "pa_lp_destroy",
           "pa_mixed_setup", "pa_mixed_apply", "pa_mixed_lumped", "pa_mixed_rk4", "pa_mixed_set_grid_cap",
           "pa_mixed_info", "pa_mixed_destroy")


class HexpaError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hexpa error {code}: {msg}")
        self.code = code


class MeshDesc(ctypes.Structure):
    _fields_ = [("nvert", ctypes.c_int32), ("vert_xyz", ctypes.c_void_p), ("nelem", ctypes.c_int32),
                ("hex", ctypes.c_void_p), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("elem_dofs", ctypes.c_void_p), ("ndof", ctypes.c_int32), ("ess_mode", ctypes.c_int32),
                ("ess_marker", ctypes.c_void_p)]


class CoeffDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("value", ctypes.c_double), ("amp", ctypes.c_double),
                ("freq", ctypes.c_double), ("grid", ctypes.c_void_p), ("gx", ctypes.c_int32),
                ("gy", ctypes.c_int32), ("gz", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("p", "q1d", "ops", "nelem", "ndof", "ness", "ncomp", "variant",
                                              "elems_per_block", "threads_per_block")] + \
               [("qdata_bytes", ctypes.c_int64), ("map_bytes", ctypes.c_int64)]


class CgOpts(ctypes.Structure):
    _fields_ = [("rtol", ctypes.c_double), ("max_it", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("constrained", ctypes.c_int32), ("lp_fmt", ctypes.c_int32),
                ("inner_max", ctypes.c_int32), ("inner_rtol", ctypes.c_double), ("lp", ctypes.c_void_p),
                ("n_capture", ctypes.c_int32), ("pad_", ctypes.c_int32), ("capture_at", ctypes.c_void_p),
                ("capture_x", ctypes.c_void_p)]


class CgResult(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("status", ctypes.c_int32), ("rel_res_recursive", ctypes.c_double),
                ("rel_res_true", ctypes.c_double), ("seconds", ctypes.c_double),
                ("inner_iters_total", ctypes.c_int32), ("fallback", ctypes.c_int32)]


class LpOpts(ctypes.Structure):
    _fields_ = [("use_net", ctypes.c_int32), ("use_coarse", ctypes.c_int32), ("coarse_iters", ctypes.c_int32),
                ("loss", ctypes.c_int32), ("seed", ctypes.c_int32), ("infer_fp16", ctypes.c_int32),
                ("lr", ctypes.c_double), ("net_scale", ctypes.c_double)]


class TrainSet(ctypes.Structure):
    _fields_ = [("ndraws", ctypes.c_int32), ("capture", ctypes.c_int32), ("ops", ctypes.c_void_p),
                ("xstar", ctypes.c_void_p), ("capture_at", ctypes.c_void_p), ("n_capture", ctypes.c_int32),
                ("epochs", ctypes.c_int32), ("seed", ctypes.c_uint32), ("pad_", ctypes.c_int32)]


class TrainLog(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int32), ("max_steps", ctypes.c_int32), ("loss", ctypes.c_void_p),
                ("seconds_capture", ctypes.c_double), ("seconds_train", ctypes.c_double)]


class MixedDesc(ctypes.Structure):
    _fields_ = [("p", ctypes.c_int32), ("pu", ctypes.c_int32), ("q1d", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("rho", ctypes.c_double), ("bulk", ctypes.c_double)]


class MixedInfo(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int32) for n in ("p", "pu", "q1d", "nelem", "ndof_p", "ndof_u", "elems_per_block",
                                              "pad_")] + [("qdata_bytes", ctypes.c_int64)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32 = ctypes.c_void_p, ctypes.c_int
    sig = {
        "pa_setup": [ctypes.POINTER(MeshDesc), i32, i32, ctypes.POINTER(CoeffDesc), ctypes.c_uint32, vp,
                     ctypes.POINTER(vp)],
        "pa_apply": [vp, vp, vp, vp],
        "pa_apply_add": [vp, vp, vp, vp],
        "pa_apply_lp": [vp, vp, vp, i32, vp],
        "pa_apply_unfused_noalloc": [vp, i32, vp, vp, vp],
        "pa_apply_constrained": [vp, vp, vp, vp],
        "pa_diag": [vp, vp, i32, vp],
        "pa_load": [vp, vp, vp, vp],
        "pa_qpoints": [vp, vp, vp],
        "pa_nodes": [vp, vp, vp],
        "pa_get_elem_dofs": [vp, vp],
        "pa_get_ess": [vp, vp],
        "pa_set_variant": [vp, i32],
        "pa_set_grid_cap": [vp, i32],
        "pa_info": [vp, ctypes.POINTER(Info)],
        "cg_solve": [vp, vp, vp, ctypes.POINTER(CgOpts), ctypes.POINTER(CgResult), vp],
        "pa_debug_mfma_f64": [i32, vp, vp, vp, vp],
        "pa_debug_mfma16": [i32, vp, vp, vp, vp],
        "pa_lp_create": [vp, ctypes.POINTER(LpOpts), ctypes.POINTER(vp)],
        "pa_lp_bind": [vp, vp],
        "pa_lp_configure": [vp, ctypes.POINTER(LpOpts)],
        "pa_lp_num_params": [],
        "pa_lp_get_params": [vp, vp, i32],
        "pa_lp_set_params": [vp, vp, i32],
        "pa_lp_logk": [vp, vp],
        "pa_lp_apply": [vp, vp, vp, vp],
        "pa_lp_coarse": [vp, vp, vp, vp],
        "pa_lp_net": [vp, vp, vp, vp],
        "pa_lp_loss_grad": [vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp, vp],
        "pa_lp_train_step": [vp, vp, vp, vp, ctypes.POINTER(ctypes.c_double), vp],
        "pa_lp_train": [vp, ctypes.POINTER(TrainSet), ctypes.POINTER(TrainLog), vp],
        "pa_mixed_setup": [ctypes.POINTER(MeshDesc), ctypes.POINTER(MixedDesc), vp, ctypes.POINTER(vp)],
        "pa_mixed_apply": [vp, vp, vp, vp, vp, vp],
        "pa_mixed_lumped": [vp, vp, vp, vp],
        "pa_mixed_rk4": [vp, vp, vp, ctypes.c_double, i32, vp],
        "pa_mixed_set_grid_cap": [vp, i32],
        "pa_mixed_info": [vp, ctypes.POINTER(MixedInfo)],
        "pa_lp_save": [vp, ctypes.c_char_p],
        "pa_lp_load": [vp, ctypes.c_char_p],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.pa_destroy.argtypes = [vp]
    lib.pa_destroy.restype = None
    lib.pa_lp_destroy.argtypes = [vp]
    lib.pa_lp_destroy.restype = None
    lib.pa_mixed_destroy.argtypes = [vp]
    lib.pa_mixed_destroy.restype = None
    lib.pa_last_error.argtypes = []
    lib.pa_last_error.restype = ctypes.c_char_p
    return lib


_lib = _load()


def lib():
    return _lib


def _check(rc, allow=()):
    if rc != PA_OK and rc not in allow:
        raise HexpaError(rc, _lib.pa_last_error().decode())
    return rc


def _dptr(t, dtype=None, n=None):
    """Device pointer of a contiguous CUDA tensor (checked)."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a CUDA (HIP) torch tensor")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected dtype {dtype}, got {t.dtype}")
    if n is not None and t.numel() != n:
        raise ValueError(f"expected {n} elements, got {t.numel()}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


# ------------------------------------------------------------------ C-ABI mirrors
def pa_setup(mesh, order, q1d, coeff=None, ops=PA_DIFFUSION, structured=True, elem_dofs=None, ndof=0,
             ess_mode=0, ess_marker=None, stream=None):
    """mesh: dict(n, vert[(nv,3)], hex[(ne,8)]).  coeff: None (=1) or dict(kind, value, amp, freq, grid)."""
    vert = np.ascontiguousarray(mesh["vert"], dtype=np.float64)
    hexes = np.ascontiguousarray(mesh["hex"], dtype=np.int32)
    md = MeshDesc()
    md.nvert, md.vert_xyz = vert.shape[0], vert.ctypes.data
    md.nelem, md.hex = hexes.shape[0], hexes.ctypes.data
    n = int(mesh.get("n", 0)) if structured else 0
    md.nx = md.ny = md.nz = n
    keep = [vert, hexes]
    if elem_dofs is not None:
        ed = np.ascontiguousarray(elem_dofs, dtype=np.int32)
        keep.append(ed)
        md.elem_dofs, md.ndof = ed.ctypes.data, int(ndof)
    md.ess_mode = int(ess_mode)
    if ess_marker is not None:
        mk = np.ascontiguousarray(ess_marker, dtype=np.uint8)
        keep.append(mk)
        md.ess_marker = mk.ctypes.data
    cd = None
    if coeff is not None:
        cd = CoeffDesc()
        cd.kind = int(coeff.get("kind", PA_COEFF_CONST))
        cd.value = float(coeff.get("value", 1.0))
        cd.amp = float(coeff.get("amp", 0.0))
        cd.freq = float(coeff.get("freq", 0.0))
        if coeff.get("grid") is not None:
            g = np.ascontiguousarray(coeff["grid"], dtype=np.float64)
            keep.append(g)
            cd.grid = g.ctypes.data
            cd.gz, cd.gy, cd.gx = g.shape
    h = ctypes.c_void_p()
    _check(_lib.pa_setup(ctypes.byref(md), int(order), int(q1d), ctypes.byref(cd) if cd is not None else None,
                         int(ops), _stream(stream), ctypes.byref(h)))
    del keep
    return h


def pa_info(h):
    info = Info()
    _check(_lib.pa_info(h, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in Info._fields_}


def pa_apply(h, x, y, stream=None):
    _check(_lib.pa_apply(h, _dptr(x), _dptr(y), _stream(stream)))


def pa_apply_add(h, x, y, stream=None):
    _check(_lib.pa_apply_add(h, _dptr(x), _dptr(y), _stream(stream)))


def pa_apply_lp(h, x, y, fmt=PA_LP_FP16, stream=None):
    import torch
    _check(_lib.pa_apply_lp(h, _dptr(x, torch.float32), _dptr(y, torch.float32), int(fmt), _stream(stream)))


def pa_apply_unfused_noalloc(h, variant, x, y, stream=None):
    _check(_lib.pa_apply_unfused_noalloc(h, int(variant), _dptr(x), _dptr(y), _stream(stream)))


def pa_apply_constrained(h, x, y, stream=None):
    _check(_lib.pa_apply_constrained(h, _dptr(x), _dptr(y), _stream(stream)))


def pa_diag(h, d, constrained=False, stream=None):
    _check(_lib.pa_diag(h, _dptr(d), int(bool(constrained)), _stream(stream)))


def pa_load(h, f_qp, b, stream=None):
    _check(_lib.pa_load(h, _dptr(f_qp), _dptr(b), _stream(stream)))


def pa_qpoints(h, xyz, stream=None):
    _check(_lib.pa_qpoints(h, _dptr(xyz), _stream(stream)))


def pa_nodes(h, xyz, stream=None):
    _check(_lib.pa_nodes(h, _dptr(xyz), _stream(stream)))


def pa_get_elem_dofs(h):
    info = pa_info(h)
    d = info["p"] + 1
    out = np.zeros((info["nelem"], d ** 3), dtype=np.int32)
    _check(_lib.pa_get_elem_dofs(h, out.ctypes.data_as(ctypes.c_void_p)))
    return out


def pa_get_ess(h):
    info = pa_info(h)
    out = np.zeros(max(info["ness"], 1), dtype=np.int32)
    _check(_lib.pa_get_ess(h, out.ctypes.data_as(ctypes.c_void_p)))
    return out[:info["ness"]]


def pa_set_variant(h, variant):
    _check(_lib.pa_set_variant(h, int(variant)))


def pa_set_grid_cap(h, max_workgroups):
    _check(_lib.pa_set_grid_cap(h, int(max_workgroups)))


def pa_destroy(h):
    _lib.pa_destroy(h)


def cg_solve(h, b, x, rtol=1e-8, max_it=10000, mode=PA_CG_JACOBI, check_every=1, constrained=True,
             lp_fmt=PA_LP_FP16, inner_max=200, inner_rtol=1e-2, lp=None, capture_at=None, capture_x=None,
             stream=None, raise_on_fail=True):
    """capture_at: ascending iteration numbers whose iterates are copied into the rows of the
    device tensor capture_x [len(capture_at)][ndof] (Jacobi-PCG only)."""
    cap = None
    o = CgOpts(float(rtol), int(max_it), int(mode), int(check_every), int(bool(constrained)), int(lp_fmt),
               int(inner_max), float(inner_rtol), None if lp is None else (lp.value if isinstance(lp, ctypes.c_void_p) else int(lp)), 0, 0, None,
               None)
    if capture_at is not None:
        cap = np.ascontiguousarray(capture_at, dtype=np.int32)
        o.n_capture = cap.size
        o.capture_at = cap.ctypes.data
        o.capture_x = _dptr(capture_x, n=cap.size * b.numel())
    r = CgResult()
    rc = _lib.cg_solve(h, _dptr(b), _dptr(x), ctypes.byref(o), ctypes.byref(r), _stream(stream))
    if raise_on_fail:
        _check(rc)
    return {"rc": rc, "iters": r.iters, "status": r.status, "rel_res_recursive": r.rel_res_recursive,
            "rel_res_true": r.rel_res_true, "seconds": r.seconds, "inner_iters_total": r.inner_iters_total,
            "fallback": r.fallback}


def _lp_opts(use_net=True, use_coarse=True, coarse_iters=4, loss=PA_LP_LOSS_ENERGY, seed=0, lr=1e-3,
             infer_fp16=True, net_scale=1.0):
    return LpOpts(int(bool(use_net)), int(bool(use_coarse)), int(coarse_iters), int(loss), int(seed),
                  int(bool(infer_fp16)), float(lr), float(net_scale))


def pa_lp_create(h, **opts):
    out = ctypes.c_void_p()
    _check(_lib.pa_lp_create(h, ctypes.byref(_lp_opts(**opts)), ctypes.byref(out)))
    return out


def pa_lp_bind(lp, h):
    _check(_lib.pa_lp_bind(lp, h))


def pa_lp_configure(lp, **opts):
    _check(_lib.pa_lp_configure(lp, ctypes.byref(_lp_opts(**opts))))


def pa_lp_num_params():
    return _lib.pa_lp_num_params()


def pa_lp_get_params(lp):
    n = pa_lp_num_params()
    out = np.zeros(n, dtype=np.float32)
    _check(_lib.pa_lp_get_params(lp, out.ctypes.data, n))
    return out


def pa_lp_set_params(lp, params):
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(_lib.pa_lp_set_params(lp, p.ctypes.data, p.size))


def pa_lp_logk(lp, out):
    _check(_lib.pa_lp_logk(lp, _dptr(out)))


def pa_lp_apply(lp, r, z, stream=None):
    _check(_lib.pa_lp_apply(lp, _dptr(r), _dptr(z), _stream(stream)))


def pa_lp_coarse(lp, r, z, stream=None):
    _check(_lib.pa_lp_coarse(lp, _dptr(r), _dptr(z), _stream(stream)))


def pa_lp_net(lp, r, z, stream=None):
    _check(_lib.pa_lp_net(lp, _dptr(r), _dptr(z), _stream(stream)))


def pa_lp_loss_grad(lp, r, t, want_grad=True, stream=None):
    loss = ctypes.c_double()
    g = np.zeros(pa_lp_num_params(), dtype=np.float32) if want_grad else None
    _check(_lib.pa_lp_loss_grad(lp, _dptr(r), _dptr(t), ctypes.byref(loss), None if g is None else g.ctypes.data,
                                _stream(stream)))
    return loss.value, g


def pa_lp_train_step(lp, b, xstar, xk, want_loss=True, stream=None):
    loss = ctypes.c_double()
    _check(_lib.pa_lp_train_step(lp, _dptr(b), _dptr(xstar), _dptr(xk), ctypes.byref(loss) if want_loss else None,
                                 _stream(stream)))
    return loss.value if want_loss else None


def pa_lp_train(lp, ops, xstars, capture_at, capture=PA_LP_CAPTURE_FCG, epochs=1, seed=0, max_steps=100000,
                stream=None):
    """ops: pa_op handles; xstars: device FP64 tensors [ndof], one per operator.  Returns
    (losses, seconds_capture, seconds_train)."""
    n = len(ops)
    opv = (ctypes.c_void_p * max(n, 1))(*[o.value if isinstance(o, ctypes.c_void_p) else o for o in ops])
    xv = (ctypes.c_void_p * max(n, 1))(*[_dptr(x).value for x in xstars])
    cat = np.ascontiguousarray(capture_at, dtype=np.int32)
    ts = TrainSet(n, int(capture), ctypes.cast(opv, ctypes.c_void_p), ctypes.cast(xv, ctypes.c_void_p),
                  cat.ctypes.data, cat.size, int(epochs), int(seed) & 0xFFFFFFFF, 0)
    loss = np.zeros(max(int(max_steps), 1))
    tl = TrainLog(0, int(max_steps), loss.ctypes.data, 0.0, 0.0)
    _check(_lib.pa_lp_train(lp, ctypes.byref(ts), ctypes.byref(tl), _stream(stream)))
    return loss[:min(tl.steps, int(max_steps))].copy(), tl.seconds_capture, tl.seconds_train


def pa_lp_save(lp, path):
    _check(_lib.pa_lp_save(lp, os.fsencode(path)))


def pa_lp_load(lp, path):
    _check(_lib.pa_lp_load(lp, os.fsencode(path)))


def pa_lp_destroy(lp):
    _lib.pa_lp_destroy(lp)


def pa_debug_mfma_f64(shape, A, B, D, stream=None):
    _check(_lib.pa_debug_mfma_f64(int(shape), _dptr(A), _dptr(B), _dptr(D), _stream(stream)))


def pa_debug_mfma16(bf16, A, B, D, stream=None):
    _check(_lib.pa_debug_mfma16(int(bool(bf16)), _dptr(A), _dptr(B), _dptr(D), _stream(stream)))


# ------------------------------------------------------------------ convenience
class PAOperator:
    """Owns a pa_op handle; thin convenience over the C calls above."""

    def __init__(self, mesh, order, q1d, coeff=None, ops=PA_DIFFUSION, ess_mode=0, **kw):
        self.h = pa_setup(mesh, order, q1d, coeff=coeff, ops=ops, ess_mode=ess_mode, **kw)
        self.info = pa_info(self.h)
        self.ndof = self.info["ndof"]
        self.nelem = self.info["nelem"]
        self.p, self.q = order, q1d

    def _vec(self, n=None):
        import torch
        return torch.empty(self.ndof if n is None else n, dtype=torch.float64, device="cuda")

    def apply(self, x, y=None):
        y = self._vec() if y is None else y
        pa_apply(self.h, x, y)
        return y

    def apply_lp(self, x32, fmt=PA_LP_FP16, y=None):
        import torch
        y = torch.empty(self.ndof, dtype=torch.float32, device="cuda") if y is None else y
        pa_apply_lp(self.h, x32, y, fmt)
        return y

    def apply_constrained(self, x, y=None):
        y = self._vec() if y is None else y
        pa_apply_constrained(self.h, x, y)
        return y

    def diag(self, constrained=False):
        d = self._vec()
        pa_diag(self.h, d, constrained)
        return d

    def qpoints(self):
        xyz = self._vec(self.nelem * self.q ** 3 * 3)
        pa_qpoints(self.h, xyz)
        return xyz.view(self.nelem, self.q ** 3, 3)

    def nodes(self):
        xyz = self._vec(self.ndof * 3)
        pa_nodes(self.h, xyz)
        return xyz.view(self.ndof, 3)

    def load(self, f_qp):
        b = self._vec()
        pa_load(self.h, f_qp.contiguous().view(-1), b)
        return b

    def set_variant(self, v):
        pa_set_variant(self.h, v)
        self.info = pa_info(self.h)

    def set_grid_cap(self, n):
        pa_set_grid_cap(self.h, n)

    def cg(self, b, x=None, **kw):
        import torch
        x = torch.zeros_like(b) if x is None else x
        res = cg_solve(self.h, b, x, **kw)
        return x, res

    def close(self):
        if self.h:
            pa_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LearnedPreconditioner:
    """Owns a pa_lp handle bound to a PAOperator (thin convenience over the pa_lp_* calls)."""

    def __init__(self, op, **opts):
        self.op = op
        self.h = pa_lp_create(op.h, **opts)

    def bind(self, op):
        pa_lp_bind(self.h, op.h)
        self.op = op

    def configure(self, **opts):
        pa_lp_configure(self.h, **opts)

    def params(self):
        return pa_lp_get_params(self.h)

    def set_params(self, p):
        pa_lp_set_params(self.h, p)

    def apply(self, r, z=None):
        z = self.op._vec() if z is None else z
        pa_lp_apply(self.h, r, z)
        return z

    def coarse(self, r, z=None):
        z = self.op._vec() if z is None else z
        pa_lp_coarse(self.h, r, z)
        return z

    def net(self, r, z=None):
        z = self.op._vec() if z is None else z
        pa_lp_net(self.h, r, z)
        return z

    def logk(self):
        import torch
        d = self.op.p + 1
        out = torch.empty(self.op.nelem * d ** 3, dtype=torch.float32, device="cuda")
        pa_lp_logk(self.h, out)
        return out

    def loss_grad(self, r, t):
        return pa_lp_loss_grad(self.h, r, t)

    def train_step(self, b, xstar, xk, want_loss=True):
        return pa_lp_train_step(self.h, b, xstar, xk, want_loss)

    def train(self, ops, xstars, capture_at, capture=PA_LP_CAPTURE_FCG, epochs=1, seed=0):
        losses, tc, tt = pa_lp_train(self.h, [o.h for o in ops], xstars, capture_at, capture, epochs, seed)
        self.op = ops[-1] if ops else self.op
        return losses, tc, tt

    def save(self, path):
        pa_lp_save(self.h, path)

    def load(self, path):
        pa_lp_load(self.h, path)

    def close(self):
        if self.h:
            pa_lp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MixedOperator:
    """Owns a pa_mixed handle: the off-diagonal blocks of the acoustic operator (thin
    convenience over the pa_mixed_* calls)."""

    def __init__(self, mesh, p=4, pu=3, q1d=5, rho=1.0, bulk=1.0, stream=None):
        vert = np.ascontiguousarray(mesh["vert"], dtype=np.float64)
        hexes = np.ascontiguousarray(mesh["hex"], dtype=np.int32)
        md = MeshDesc()
        md.nvert, md.vert_xyz = vert.shape[0], vert.ctypes.data
        md.nelem, md.hex = hexes.shape[0], hexes.ctypes.data
        md.nx = md.ny = md.nz = int(mesh["n"])
        desc = MixedDesc(int(p), int(pu), int(q1d), 0, float(rho), float(bulk))
        h = ctypes.c_void_p()
        _check(_lib.pa_mixed_setup(ctypes.byref(md), ctypes.byref(desc), _stream(stream), ctypes.byref(h)))
        self.h = h
        info = MixedInfo()
        _check(_lib.pa_mixed_info(h, ctypes.byref(info)))
        self.info = {f: getattr(info, f) for f, _ in MixedInfo._fields_ if f != "pad_"}
        self.ndof_p, self.ndof_u, self.nelem = info.ndof_p, info.ndof_u, info.nelem
        self.nu = (int(pu) + 1) ** 3

    def _vec(self, n):
        import torch
        return torch.empty(n, dtype=torch.float64, device="cuda")

    def apply(self, u, p, yu=None, yp=None, stream=None):
        yu = self._vec(self.ndof_u) if yu is None else yu
        yp = self._vec(self.ndof_p) if yp is None else yp
        _check(_lib.pa_mixed_apply(self.h, _dptr(u, n=self.ndof_u), _dptr(p, n=self.ndof_p),
                                   _dptr(yu, n=self.ndof_u), _dptr(yp, n=self.ndof_p), _stream(stream)))
        return yu, yp

    def lumped(self, stream=None):
        mu = self._vec(self.nelem * self.nu)
        mp = self._vec(self.ndof_p)
        _check(_lib.pa_mixed_lumped(self.h, _dptr(mu), _dptr(mp), _stream(stream)))
        return mu, mp

    def rk4(self, u, p, dt, nsteps, stream=None):
        _check(_lib.pa_mixed_rk4(self.h, _dptr(u, n=self.ndof_u), _dptr(p, n=self.ndof_p), float(dt), int(nsteps),
                                 _stream(stream)))

    def set_grid_cap(self, n):
        _check(_lib.pa_mixed_set_grid_cap(self.h, int(n)))

    def close(self):
        if self.h:
            _lib.pa_mixed_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
