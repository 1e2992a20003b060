"""Mixed precision on MI355X: the 16-bit-MFMA inner apply and FP64 iterative refinement.

Bars.  The 16-bit apply is not expected to match the FP64 oracle to rounding: every
element tile and intermediate tensor is rounded to FP16 (unit roundoff u = 2^-11) or BF16
(u = 2^-8) before it enters an MFMA.  Six roundings along the contraction chain with
FP32 accumulation give a normwise relative error of a few u for rough inputs; the bounds
below are 8u (FP16: 3.9e-3) and 8u (BF16: 3.1e-2): real indexing or scaling errors show
at O(1), rounding stays a small multiple of u.  The solver is
judged in FP64: its true residual, recomputed by the CPU oracle's operator, must meet the
requested 1e-10.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import solvers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hx():
    import torch  # noqa: F401
    from paper_2603_09038_amd import hexpa
    return hexpa


def _t(a, dtype=None):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda")


def _round16(a, bf16):
    a = np.asarray(a, dtype=np.float32)
    if not bf16:
        return a.astype(np.float16).astype(np.float64)
    u = a.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("bf16", [False, True])
def test_mfma_16bit_lane_layouts(hx, bf16):
    import torch
    rng = np.random.default_rng(8)
    A = rng.integers(-8, 9, (16, 16)).astype(np.float32)  # exact in FP16 and BF16
    B = rng.integers(-8, 9, (16, 16)).astype(np.float32)
    raw = torch.zeros(256, dtype=torch.float32, device="cuda")
    hx.pa_debug_mfma16(bf16, _t(A, torch.float32), _t(B, torch.float32), raw)
    raw = raw.cpu().numpy().reshape(64, 4)
    D = A.astype(np.float64) @ B.astype(np.float64)
    for l in range(64):
        for v in range(4):
            assert raw[l, v] == D[4 * (l // 16) + v, l % 16], (l, v)
    # rounding of non-representable inputs: the product of the rounded operands
    A = rng.standard_normal((16, 16)).astype(np.float32)
    B = rng.standard_normal((16, 16)).astype(np.float32)
    raw = torch.zeros(256, dtype=torch.float32, device="cuda")
    hx.pa_debug_mfma16(bf16, _t(A, torch.float32), _t(B, torch.float32), raw)
    raw = raw.cpu().numpy().reshape(64, 4)
    D = _round16(A, bf16) @ _round16(B, bf16)
    got = np.zeros((16, 16))
    for l in range(64):
        for v in range(4):
            got[4 * (l // 16) + v, l % 16] = raw[l, v]
    np.testing.assert_allclose(got, D, rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("p,ops", [(2, 2), (4, 2), (6, 2), (4, 1), (3, 3), (8, 2)])
@pytest.mark.parametrize("fmt", [0, 1])
def test_lp_apply_accuracy(hx, p, ops, fmt):
    import torch
    n = {2: 5, 3: 4, 4: 3, 6: 2, 8: 2}[p]
    mesh = synth.box_mesh(n, perturb=0.1, seed=p)
    grid, _ = synth.lognormal_kappa_grid(1, sigma=1.0, ell=0.1, nfft=32)
    op = hx.PAOperator(mesh, p, p + 2, coeff={"kind": hx.PA_COEFF_GRID, "grid": grid}, ops=ops)
    x = synth.rand_x(op.ndof, 5)
    P = oracle.Problem(mesh, p, p + 2, coeff=oracle.Coeff.from_grid(grid),
                       ops=(oracle.MASS if ops & 1 else 0) | (oracle.DIFFUSION if ops & 2 else 0))
    ref = P.apply(x)
    y = op.apply_lp(_t(x, torch.float32), fmt=fmt).double().cpu().numpy()
    err = np.linalg.norm(y - ref) / np.linalg.norm(ref)
    u = 2.0 ** -11 if fmt == 0 else 2.0 ** -8
    assert err <= 8 * u, (p, ops, fmt, err)
    # the FP64 path on the same operator is unaffected
    y64 = op.apply(_t(x)).cpu().numpy()
    assert np.linalg.norm(y64 - ref) / np.linalg.norm(ref) <= 1e-12
    op.close()


@pytest.mark.parametrize("p", [4, 6])
def test_bf16_diffusion_apply_ignores_constants(hx, p):
    """The BF16 diffusion apply centres every element tile on its mean before rounding
    (diffusion annihilates constants element by element), so adding a constant to x changes
    the result only through FP32 rounding of the shifted input; an uncentred BF16 tile would
    carry an error of about u_bf16 times the constant (here O(1) relative)."""
    import torch
    n = {4: 3, 6: 2}[p]  # register-staged kernel at p = 4, direct-to-LDS kernel at p = 6
    mesh = synth.box_mesh(n, perturb=0.1, seed=p)
    op = hx.PAOperator(mesh, p, p + 2, ops=hx.PA_DIFFUSION)
    x = synth.rand_x(op.ndof, 3)
    y0 = op.apply_lp(_t(x, torch.float32), fmt=1).double().cpu().numpy()
    y1 = op.apply_lp(_t(x + 64.0, torch.float32), fmt=1).double().cpu().numpy()
    rel = np.linalg.norm(y1 - y0) / np.linalg.norm(y0)
    assert rel <= 1e-2, (p, rel)
    ref = oracle.Problem(mesh, p, p + 2, ops=oracle.DIFFUSION).apply(x)
    assert np.linalg.norm(y1 - ref) / np.linalg.norm(ref) <= 8 * 2.0 ** -8
    op.close()


@pytest.mark.parametrize("outer,fmt", [("ir", 0), ("ir", 1), ("fcg", 0), ("fcg", 1), ("ru", 0), ("ru", 1)])
def test_mixed_ir_reaches_fp64_tolerance(hx, fmt, outer):
    """Log-normal coefficient (sigma = 1, correlation length 0.1), p = 6, Q = 8, Dirichlet,
    b = A_c x* with x* the nodal interpolant of sin(pi x) sin(pi y) sin(pi z)."""
    import torch
    n, p, q = 4, 6, 8
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    grid, contrast = synth.lognormal_kappa_grid(0, sigma=1.0, ell=0.1, nfft=64)
    op = hx.PAOperator(mesh, p, q, coeff={"kind": hx.PA_COEFF_GRID, "grid": grid}, ops=2, ess_mode=1)
    xs = synth.u_manufactured(op.nodes().cpu().numpy())
    b = op.apply_constrained(_t(xs))
    x = torch.zeros_like(b)
    if outer == "ru":  # reliable updates: max_it bounds the total iterations, inner_max the period
        res = hx.cg_solve(op.h, b, x, rtol=1e-10, max_it=3000, mode=hx.PA_CG_MIXED_RU, lp_fmt=fmt, inner_max=40)
    else:
        mode = hx.PA_CG_MIXED_IR if outer == "ir" else hx.PA_CG_MIXED_FCG
        res = hx.cg_solve(op.h, b, x, rtol=1e-10, max_it=60, mode=mode, lp_fmt=fmt, inner_rtol=1e-2, inner_max=400)
    assert res["rc"] == 0 and res["rel_res_true"] <= 1e-10, res
    P = oracle.Problem(mesh, p, q, coeff=oracle.Coeff.from_grid(grid), ops=oracle.DIFFUSION)
    Ac = solvers.constrained(P.apply, oracle.box_boundary(n, p).astype(bool))
    bb, xx = b.cpu().numpy(), x.cpu().numpy()
    assert np.linalg.norm(bb - Ac(xx)) <= 1.05e-10 * np.linalg.norm(bb)
    assert np.linalg.norm(xx - xs) <= 1e-7 * np.linalg.norm(xs)
    # FP64 Jacobi-PCG on the same system for reference
    x64 = torch.zeros_like(b)
    r64 = hx.cg_solve(op.h, b, x64, rtol=1e-10, max_it=5000, mode=hx.PA_CG_JACOBI)
    assert r64["rc"] == 0
    assert res["inner_iters_total"] <= 3 * r64["iters"], (res, r64)
    op.close()
