"""Parity of the HIP path (through the C-ABI) against the CPU oracle, on MI355X.

Bars: index maps bit-exact; FP64 apply/diag/load within 1e-12 relative in the 2-norm
and the max-norm (the operator reaches the plain element-assembly result up to
rounding order; 1e-12 leaves ~1e3-1e4 ulps of headroom for the different summation
orders of sum factorization, MFMA accumulation and atomics).
"""
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


def _cuda(a):
    import torch
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return max(np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max())


def _ops_o(ops):
    return (oracle.MASS if ops & 1 else 0) | (oracle.DIFFUSION if ops & 2 else 0)


def test_mfma_f64_4x4x4_lane_layout(hx):
    """v_mfma_f64_4x4x4f64 (the apply kernels' MFMA): block b = (l>>2)&3 reads A[b][l&3][l>>4],
    B[b][l>>4][l&3] and lane l returns D[b][l>>4][l&3] — pinned with operands that make every
    product entry distinct, then with random operands against a CPU product."""
    import torch
    raw = torch.zeros(64, dtype=torch.float64, device="cuda")
    # D[b][i][j] = j + 10 i + 100 b + 1000 (via k = 0 and k = 1 terms)
    A = np.zeros((4, 4, 4))
    B = np.zeros((4, 4, 4))
    for b in range(4):
        A[b, :, 0] = 1.0
        A[b, :, 1] = np.arange(4)
        B[b, 0, :] = np.arange(4) + 100 * b + 1000
        B[b, 1, :] = 10.0
    hx.pa_debug_mfma_f64(4, _cuda(A.ravel()), _cuda(B.ravel()), raw)
    raw = raw.cpu().numpy()
    lanes = np.arange(64)
    expect = (lanes & 3) + 10 * (lanes >> 4) + 100 * ((lanes >> 2) & 3) + 1000
    assert np.array_equal(raw, expect.astype(float)), raw.reshape(4, 16)
    rng = np.random.default_rng(4)
    A = rng.standard_normal((4, 4, 4))
    B = rng.standard_normal((4, 4, 4))
    hx.pa_debug_mfma_f64(4, _cuda(A.ravel()), _cuda(B.ravel()), raw := torch.zeros(64, dtype=torch.float64,
                                                                                  device="cuda"))
    raw = raw.cpu().numpy()
    D = np.einsum("bik,bkj->bij", A, B)
    got = np.zeros((4, 4, 4))
    for l in range(64):
        got[(l >> 2) & 3, l >> 4, l & 3] = raw[l]
    np.testing.assert_allclose(got, D, rtol=1e-14, atol=1e-14)


def test_mfma_f64_16x16x4_lane_layout(hx):
    """v_mfma_f64_16x16x4f64 against a CPU GEMM: lane l, element v holds D[l/16 + 4v][l%16]."""
    import torch
    # structured operands: D[i][j] = j + 1000 i identifies every entry
    A = np.zeros((16, 4))
    A[:, 0], A[:, 1] = 1.0, np.arange(16)
    B = np.zeros((4, 16))
    B[0, :], B[1, :] = np.arange(16), 1000.0
    raw = torch.zeros(256, dtype=torch.float64, device="cuda")
    hx.pa_debug_mfma_f64(16, _cuda(A.ravel()), _cuda(B.ravel()), raw)
    raw = raw.cpu().numpy().reshape(64, 4)
    held = {(int(v) // 1000, int(v) % 1000) for v in raw.ravel()}
    assert len(held) == 256  # every entry of D exactly once
    rows, cols = raw // 1000, raw % 1000
    lanes = np.arange(64)
    assert np.array_equal(cols, np.repeat((lanes % 16)[:, None], 4, 1)), cols[::16]
    expect = (lanes // 16)[:, None] + 4 * np.arange(4)[None, :]
    assert np.array_equal(rows, expect), f"rows held by lanes 0,16,32,48: {rows[::16].tolist()}"
    # random operands: the same map reproduces A @ B
    rng = np.random.default_rng(3)
    A = rng.standard_normal((16, 4))
    B = rng.standard_normal((4, 16))
    hx.pa_debug_mfma_f64(16, _cuda(A.ravel()), _cuda(B.ravel()), raw := torch.zeros(256, dtype=torch.float64,
                                                                                 device="cuda"))
    raw = raw.cpu().numpy().reshape(64, 4)
    D = np.zeros((16, 16))
    for l in range(64):
        for v in range(4):
            D[l // 16 + 4 * v, l % 16] = raw[l, v]
    np.testing.assert_allclose(D, A @ B, rtol=1e-14, atol=1e-14)


@pytest.mark.parametrize("n,p", [(4, 2), (3, 4), (2, 7)])
def test_maps_bit_exact(hx, n, p):
    mesh = synth.box_mesh(n)
    op = hx.PAOperator(mesh, p, p + 2, ess_mode=1)
    assert np.array_equal(hx.pa_get_elem_dofs(op.h), oracle.box_elem_dofs(n, p))
    assert np.array_equal(hx.pa_get_ess(op.h), np.nonzero(oracle.box_boundary(n, p))[0].astype(np.int32))
    op.close()


@pytest.mark.parametrize("ops", [1, 2, 3])
def test_c1_parity(hx, ops):
    """4^3 perturbed unit cube, p=2, 4^3 Gauss points, kappa = 1, x ~ U[-1,1]: 729 DOFs."""
    mesh = synth.box_mesh(4, perturb=0.1, seed=0)
    op = hx.PAOperator(mesh, 2, 4, ops=ops)
    assert op.ndof == 729
    x = synth.rand_x(op.ndof, 0)
    ref = oracle.Problem(mesh, 2, 4, ops=_ops_o(ops)).apply(x)
    for variant in (hx.PA_VARIANT_MFMA, hx.PA_VARIANT_VALU, hx.PA_VARIANT_MFMA_COLORED, hx.PA_VARIANT_MFMA_UNFUSED,
                    hx.PA_VARIANT_VALU_UNFUSED, hx.PA_VARIANT_MFMA_MF, hx.PA_VARIANT_VALU_MF):
        op.set_variant(variant)
        y = op.apply(_cuda(x)).cpu().numpy()
        assert _rel(y, ref) <= TOL, (variant, _rel(y, ref))
    op.close()


# several element groups and a ragged tail at every order (n^3 is never a multiple of
# the elements-per-workgroup count except by accident), both quadrature sizes
@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("dq", [1, 2])
def test_apply_parity_orders(hx, p, dq):
    q = p + dq
    n = {1: 7, 2: 5, 3: 4, 4: 3, 5: 3, 6: 2, 7: 2, 8: 2}[p]
    mesh = synth.box_mesh(n, perturb=0.1, seed=p)
    coeff = {"kind": hx.PA_COEFF_SINE, "value": 1.0, "amp": 0.5, "freq": 2.0}
    for ops in (1, 2, 3):
        op = hx.PAOperator(mesh, p, q, coeff=coeff, ops=ops)
        x = synth.rand_x(op.ndof, p)
        ref = oracle.Problem(mesh, p, q, coeff=oracle.Coeff.sine(), ops=_ops_o(ops)).apply(x)
        for variant in (hx.PA_VARIANT_MFMA, hx.PA_VARIANT_VALU, hx.PA_VARIANT_MFMA_UNFUSED,
                        hx.PA_VARIANT_VALU_UNFUSED, hx.PA_VARIANT_MFMA_MF, hx.PA_VARIANT_VALU_MF):
            op.set_variant(variant)
            y = op.apply(_cuda(x)).cpu().numpy()
            assert _rel(y, ref) <= TOL, (p, q, ops, variant, _rel(y, ref))
        op.close()


# The persistent path at the stated bar.  Large meshes give every workgroup several element
# groups, and with them the cross-group pipeline: the next group's DOF map and x gathered
# (into registers, or straight into LDS by the DMA kernels at p >= 5, with their triple-
# buffered maps) and its D loaded while the current group is contracted, and LDS reused
# behind the last barrier.  A grid cap gives small meshes the same walk: 8 workgroups (one
# per XCD, each walking its XCD's contiguous range of groups), 3 (plain striding over all
# groups), both with at least three groups per workgroup, and 13 (uneven: XCDs 0..4 hold
# two workgroups, 5..7 one).  Full vectors against the oracle, 2-norm and max-norm.
MULTI = {1: 12, 2: 10, 3: 10, 4: 8, 5: 7, 6: 6, 7: 5, 8: 4}


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_persistent_multigroup_full_vector(hx, p):
    n, q = MULTI[p], p + 2
    mesh = synth.box_mesh(n, perturb=0.1, seed=100 + p)
    coeff = {"kind": hx.PA_COEFF_SINE, "value": 1.0, "amp": 0.5, "freq": 2.0}
    for ops in (1, 2, 3):
        op = hx.PAOperator(mesh, p, q, coeff=coeff, ops=ops)
        x = synth.rand_x(op.ndof, 100 + p)
        ref = oracle.Problem(mesh, p, q, coeff=oracle.Coeff.sine(), ops=_ops_o(ops)).apply(x)
        xd = _cuda(x)
        for variant in (hx.PA_VARIANT_MFMA, hx.PA_VARIANT_VALU, hx.PA_VARIANT_MFMA_UNFUSED,
                        hx.PA_VARIANT_VALU_UNFUSED, hx.PA_VARIANT_MFMA_MF, hx.PA_VARIANT_VALU_MF):
            op.set_variant(variant)
            ngroups = -(-op.nelem // op.info["elems_per_block"])
            for cap in (8, 3, 13):
                if cap != 13:
                    assert ngroups >= 3 * cap, (p, ops, variant, ngroups, cap)
                op.set_grid_cap(cap)
                y = op.apply(xd).cpu().numpy()
                assert _rel(y, ref) <= TOL, (p, ops, variant, cap, _rel(y, ref))
            op.set_grid_cap(0)
        op.close()


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_unstructured_element_order_full_vector(hx, p):
    """The same operator with its elements listed in a random order and in reverse order
    (an unstructured mesh: explicit element-to-DOF map).  Consecutive elements of a group are
    then rarely x-neighbours, or neighbours on the other side, so the scatter's shared-face
    merge mostly finds nothing to merge and the row-order gather reads scattered DOFs.  Full
    vectors against the oracle (given the same element order) at 1e-12, uncapped and with each
    workgroup walking several groups."""
    n, q = MULTI[p], p + 2
    mesh = synth.box_mesh(n, perturb=0.1, seed=140 + p)
    ed = oracle.box_elem_dofs(n, p)
    ndof = int(ed.max()) + 1
    perm = np.random.default_rng(140 + p).permutation(n ** 3)
    x = synth.rand_x(ndof, 140 + p)
    xd = _cuda(x)
    for order in (perm, np.arange(n ** 3)[::-1]):
        m2 = {"vert": mesh["vert"], "hex": np.ascontiguousarray(mesh["hex"][order])}
        ed2 = np.ascontiguousarray(ed[order])
        for ops in (1, 2):
            ref = oracle.Problem(m2, p, q, ops=_ops_o(ops), elem_dofs=ed2).apply(x)
            op = hx.PAOperator(m2, p, q, ops=ops, structured=False, elem_dofs=ed2, ndof=ndof)
            assert op.ndof == ndof
            for variant in (hx.PA_VARIANT_MFMA, hx.PA_VARIANT_VALU):
                op.set_variant(variant)
                for cap in (0, 3):
                    op.set_grid_cap(cap)
                    y = op.apply(xd).cpu().numpy()
                    assert _rel(y, ref) <= TOL, (p, ops, variant, cap, _rel(y, ref))
                    assert np.max(np.abs(y - ref)) <= TOL * np.max(np.abs(ref)), (p, ops, variant, cap)
            op.close()


@pytest.mark.parametrize("p", [2, 4, 6, 8])
def test_persistent_multigroup_lp_apply(hx, p):
    """The 16-bit apply on the same multi-group walk: within 8u of the FP64 oracle, and
    equal (up to the FP32 atomic order) to the uncapped launch."""
    import torch
    n, q = MULTI[p], p + 2
    mesh = synth.box_mesh(n, perturb=0.1, seed=120 + p)
    op = hx.PAOperator(mesh, p, q, ops=2)
    x = synth.rand_x(op.ndof, 120 + p)
    ref = oracle.Problem(mesh, p, q, ops=oracle.DIFFUSION).apply(x)
    x32 = torch.tensor(x, dtype=torch.float32, device="cuda")
    for fmt, u in ((hx.PA_LP_FP16, 2.0 ** -11), (hx.PA_LP_BF16, 2.0 ** -8)):
        y0 = op.apply_lp(x32, fmt=fmt).double().cpu().numpy()
        for cap in (8, 3):
            op.set_grid_cap(cap)
            y = op.apply_lp(x32, fmt=fmt).double().cpu().numpy()
            op.set_grid_cap(0)
            assert _rel(y, ref) <= 8 * u, (p, fmt, cap, _rel(y, ref))
            assert _rel(y, y0) <= 1e-5, (p, fmt, cap, _rel(y, y0))
    op.close()


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5, 6, 7, 8])
def test_diag_parity_orders(hx, p):
    """The sum-factorised diagonal against the oracle's diagonal of the dense element
    matrices, every operator combination, both quadrature sizes, plain and constrained."""
    from oracle import solvers
    n = {1: 5, 2: 4, 3: 3, 4: 3, 5: 2, 6: 2, 7: 2, 8: 2}[p]
    mesh = synth.box_mesh(n, perturb=0.1, seed=30 + p)
    coeff = {"kind": hx.PA_COEFF_SINE, "value": 1.0, "amp": 0.5, "freq": 2.0}
    ess = oracle.box_boundary(n, p).astype(bool)
    for q in (p + 1, p + 2):
        for ops in (1, 2, 3):
            op = hx.PAOperator(mesh, p, q, coeff=coeff, ops=ops, ess_mode=1)
            ref = oracle.Problem(mesh, p, q, coeff=oracle.Coeff.sine(), ops=_ops_o(ops)).diag()
            assert _rel(op.diag().cpu().numpy(), ref) <= TOL, (p, q, ops)
            dc = op.diag(constrained=True).cpu().numpy()
            assert _rel(dc, solvers.constrained_diag(ref, ess)) <= TOL, (p, q, ops)
            op.close()


def test_grid_coefficient_and_diag_load_points(hx):
    p, q, n = 3, 5, 3
    mesh = synth.box_mesh(n, perturb=0.1, seed=9)
    grid, _ = synth.lognormal_kappa_grid(4, sigma=1.0, ell=0.1, nfft=32)
    op = hx.PAOperator(mesh, p, q, coeff={"kind": hx.PA_COEFF_GRID, "grid": grid}, ops=3, ess_mode=1)
    P = oracle.Problem(mesh, p, q, coeff=oracle.Coeff.from_grid(grid), ops=3)
    x = synth.rand_x(op.ndof, 2)
    assert _rel(op.apply(_cuda(x)).cpu().numpy(), P.apply(x)) <= TOL
    for variant in (hx.PA_VARIANT_MFMA_MF, hx.PA_VARIANT_VALU_MF):  # D recomputed from the grid coefficient
        op.set_variant(variant)
        assert _rel(op.apply(_cuda(x)).cpu().numpy(), P.apply(x)) <= TOL, variant
    op.set_variant(hx.PA_VARIANT_MFMA)
    assert _rel(op.diag().cpu().numpy(), P.diag()) <= TOL
    xq = op.qpoints().cpu().numpy()
    np.testing.assert_allclose(xq, P.qpoints(), rtol=0, atol=1e-15)
    np.testing.assert_allclose(op.nodes().cpu().numpy(), P.nodes(), rtol=0, atol=1e-15)
    fq = synth.f_manufactured(xq.reshape(-1, 3)).reshape(P.nelem, -1)
    assert _rel(op.load(_cuda(fq)).cpu().numpy(), P.load(fq)) <= TOL
    # constrained apply / diag
    ess = oracle.box_boundary(n, p).astype(bool)
    from oracle import solvers
    yc = op.apply_constrained(_cuda(x)).cpu().numpy()
    assert _rel(yc, solvers.constrained(P.apply, ess)(x)) <= TOL
    dc = op.diag(constrained=True).cpu().numpy()
    assert _rel(dc, solvers.constrained_diag(P.diag(), ess)) <= TOL
    op.close()


def test_single_element_reconstructs_element_matrix(hx):
    """n = 1: applying to unit vectors rebuilds A_e column by column."""
    mesh = synth.box_mesh(1)
    rng = np.random.default_rng(5)
    mesh["vert"] = mesh["vert"] + rng.uniform(-0.1, 0.1, mesh["vert"].shape)
    p, q = 3, 5
    op = hx.PAOperator(mesh, p, q, ops=3)
    Ae = oracle.Problem(mesh, p, q, ops=3).elem_matrices()[0]
    import torch
    I = torch.eye(op.ndof, dtype=torch.float64, device="cuda")
    cols = np.stack([op.apply(I[k].contiguous()).cpu().numpy() for k in range(op.ndof)], 1)
    assert np.abs(cols - Ae).max() <= TOL * np.abs(Ae).max()
    op.close()


def test_coloured_apply_is_bitwise_reproducible(hx):
    mesh = synth.box_mesh(6, perturb=0.1, seed=1)
    op = hx.PAOperator(mesh, 4, 6, ops=2)
    op.set_variant(hx.PA_VARIANT_MFMA_COLORED)
    x = _cuda(synth.rand_x(op.ndof, 3))
    y1 = op.apply(x).cpu().numpy()
    y2 = op.apply(x).cpu().numpy()
    assert np.array_equal(y1, y2)
    op.set_variant(hx.PA_VARIANT_MFMA)
    assert _rel(op.apply(x).cpu().numpy(), y1) <= TOL
    op.close()


def test_jacobi_pcg_true_residual_under_oracle(hx):
    """C2-shaped problem at reduced size: sine coefficient, manufactured RHS, Dirichlet."""
    n, p, q = 6, 4, 6
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    coeff = {"kind": hx.PA_COEFF_SINE, "value": 1.0, "amp": 0.5, "freq": 2.0}
    op = hx.PAOperator(mesh, p, q, coeff=coeff, ops=2, ess_mode=1)
    xq = op.qpoints().cpu().numpy().reshape(-1, 3)
    b = op.load(_cuda(synth.f_manufactured(xq).reshape(op.nelem, -1)))
    ess = hx.pa_get_ess(op.h)
    import torch
    b[torch.tensor(ess, device="cuda", dtype=torch.long)] = 0.0
    x, res = op.cg(b, rtol=1e-8, max_it=2000, mode=hx.PA_CG_JACOBI)
    assert res["rc"] == 0 and res["rel_res_true"] <= 1e-8
    # judged by the oracle operator
    P = oracle.Problem(mesh, p, q, coeff=oracle.Coeff.sine(), ops=oracle.DIFFUSION)
    from oracle import solvers
    essm = oracle.box_boundary(n, p).astype(bool)
    Ac = solvers.constrained(P.apply, essm)
    bb = b.cpu().numpy()
    xx = x.cpu().numpy()
    assert np.linalg.norm(bb - Ac(xx)) <= 1.01e-8 * np.linalg.norm(bb)
    # iteration count close to the oracle's PCG on the same system
    dinv = 1.0 / solvers.constrained_diag(P.diag(), essm)
    _, it_o, _, _, _ = solvers.pcg(Ac, bb, lambda r: dinv * r, rtol=1e-8)
    assert abs(res["iters"] - it_o) <= 2 + 0.02 * it_o, (res["iters"], it_o)
    op.close()


def _sample_rows(ndof, seed, k=2000):
    return np.unique(np.concatenate([np.random.default_rng(seed).integers(0, ndof, k), [0, ndof - 1]]))


def _linear_nodal(P, a=(0.3, -0.7, 0.5), b=0.25):
    """Nodal values of u(x) = a.x + b.  The trilinear map makes x a polynomial of degree <= 1
    per reference direction, so u lies in the discrete space on any perturbed mesh."""
    return P.nodes() @ np.asarray(a) + b


def _check_linear(y_lin, interior, scale, ops, a=(0.3, -0.7, 0.5), b=0.25, u=None):
    """Diffusion with kappa = 1: (K u)_i = integral of a . grad phi_i, which vanishes for every
    node i off the boundary (divergence theorem; the Gauss rule with Q = p + 2 integrates
    a . adj(J)^T grad phi exactly).  Mass: u^T M u = integral of u^2 over the unit cube.
    Both fail on a gather or scatter index error, unlike K 1 = 0."""
    if ops == 2:
        assert np.abs(y_lin[interior]).max() <= TOL * scale, np.abs(y_lin[interior]).max() / scale
    else:
        a1, a2, a3 = a
        exact = (a1 * a1 + a2 * a2 + a3 * a3) / 3 + (a1 * a2 + a1 * a3 + a2 * a3) / 2 + b * (a1 + a2 + a3) + b * b
        assert abs(float(u @ y_lin) - exact) <= TOL * exact * 10, (float(u @ y_lin), exact)


def test_full_size_c2_sampled_rows(hx):
    """48^3 perturbed mesh, p=4, Q=6, sine coefficient (7,189,057 DOFs), in the launch
    configuration the benchmark times: 2000 sampled rows against the oracle's row evaluation
    at the stated bar (max-norm over the rows relative to their largest entry)."""
    n, p, q = 48, 4, 6
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    coeff = {"kind": hx.PA_COEFF_SINE, "value": 1.0, "amp": 0.5, "freq": 2.0}
    op = hx.PAOperator(mesh, p, q, coeff=coeff, ops=2)
    assert op.ndof == 7189057
    x = synth.rand_x(op.ndof, 0)
    y = op.apply(_cuda(x)).cpu().numpy()
    rows = _sample_rows(op.ndof, 0)
    P = oracle.Problem(mesh, p, q, coeff=oracle.Coeff.sine(), ops=oracle.DIFFUSION)
    ref = P.apply_rows(x, rows)
    scale = np.abs(ref).max()
    err = np.abs(y[rows] - ref).max() / scale
    print(f"C2 sampled rows: max error / scale {err:.2e} over {rows.size} rows")
    assert err <= TOL
    assert np.linalg.norm(y[rows] - ref) <= TOL * np.linalg.norm(ref)
    # property at any size: K 1 = 0 (the sine coefficient rules out the linear-function check)
    import torch
    one = torch.ones(op.ndof, dtype=torch.float64, device="cuda")
    assert float(op.apply(one).abs().max()) <= 1e-12 * scale
    op.close()


# the order sweep at its full sizes (about 30 M DOFs each), default kernel choice
@pytest.mark.parametrize("n,p", [(155, 2), (78, 4), (52, 6), (40, 8)])
@pytest.mark.parametrize("ops", [1, 2])
def test_full_size_sweep_sampled_rows(hx, n, p, ops):
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    op = hx.PAOperator(mesh, p, p + 2, ops=ops)
    assert op.ndof == (n * p + 1) ** 3
    x = synth.rand_x(op.ndof, 0)
    y = op.apply(_cuda(x)).cpu().numpy()
    rows = _sample_rows(op.ndof, p)
    P = oracle.Problem(mesh, p, p + 2, ops=_ops_o(ops))
    ref = P.apply_rows(x, rows)
    scale = np.abs(ref).max()
    err = np.abs(y[rows] - ref).max() / scale
    print(f"n={n} p={p} ops={ops}: max error / scale {err:.2e} over {rows.size} rows")
    assert err <= TOL, (n, p, ops, err)
    assert np.linalg.norm(y[rows] - ref) <= TOL * np.linalg.norm(ref)
    # properties over the whole vector, at any size, sensitive to index errors
    u = _linear_nodal(P)
    y_lin = op.apply(_cuda(u)).cpu().numpy()
    interior = ~oracle.box_boundary(n, p).astype(bool)
    _check_linear(y_lin, interior, scale, ops, u=u)
    op.close()


def test_full_size_mixed_workload_lp_apply_sampled_rows(hx):
    """32^3, p=6, Q=8, log-normal coefficient (7,189,057 DOFs): the 16-bit apply on sampled
    rows against the oracle, max-norm over the rows within 16u of the rows' scale."""
    import torch
    n, p, q = 32, 6, 8
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    grid, _ = synth.lognormal_kappa_grid(0, sigma=1.0, ell=0.1)
    op = hx.PAOperator(mesh, p, q, coeff={"kind": hx.PA_COEFF_GRID, "grid": grid}, ops=2)
    x = synth.rand_x(op.ndof, 0)
    rows = np.unique(np.concatenate([np.random.default_rng(6).integers(0, op.ndof, 48), [0, op.ndof - 1]]))
    ref = oracle.Problem(mesh, p, q, coeff=oracle.Coeff.from_grid(grid), ops=oracle.DIFFUSION).apply_rows(x, rows)
    scale = np.abs(ref).max()
    x32 = torch.tensor(x, dtype=torch.float32, device="cuda")
    for fmt, u in ((hx.PA_LP_FP16, 2.0 ** -11), (hx.PA_LP_BF16, 2.0 ** -8)):
        y = op.apply_lp(x32, fmt=fmt).double().cpu().numpy()
        assert np.abs(y[rows] - ref).max() <= 16 * u * scale, (fmt, np.abs(y[rows] - ref).max() / scale)
    op.close()


def test_zero_input_and_zero_right_hand_side(hx):
    """Degenerate inputs: A 0 = 0 exactly for every variant; b = 0 returns x = 0 exactly, with
    no iteration, for every solver mode (a nonzero initial guess is overwritten); FCG without
    a preconditioner handle is still rejected."""
    import torch
    mesh = synth.box_mesh(3, perturb=0.1, seed=4)
    for ops in (1, 2, 3):
        op = hx.PAOperator(mesh, 2, 4, ops=ops, ess_mode=1)
        z = torch.zeros(op.ndof, dtype=torch.float64, device="cuda")
        for variant in (hx.PA_VARIANT_MFMA, hx.PA_VARIANT_VALU, hx.PA_VARIANT_MFMA_COLORED,
                        hx.PA_VARIANT_MFMA_UNFUSED, hx.PA_VARIANT_VALU_UNFUSED, hx.PA_VARIANT_MFMA_MF,
                        hx.PA_VARIANT_VALU_MF):
            op.set_variant(variant)
            y = op.apply(z)
            assert torch.count_nonzero(y).item() == 0, (ops, variant)
        op.set_variant(hx.PA_VARIANT_MFMA)
        if ops == 2:
            for mode in (hx.PA_CG_PLAIN, hx.PA_CG_JACOBI, hx.PA_CG_MIXED_IR, hx.PA_CG_MIXED_FCG, hx.PA_CG_MIXED_RU):
                x = _cuda(synth.rand_x(op.ndof, 1))
                r = hx.cg_solve(op.h, z, x, rtol=1e-8, max_it=50, mode=mode)
                assert r["rc"] == 0 and r["iters"] == 0, (mode, r)
                assert torch.count_nonzero(x).item() == 0, mode
            x = torch.zeros_like(z)
            r = hx.cg_solve(op.h, z, x, mode=hx.PA_CG_FCG, raise_on_fail=False)
            assert r["rc"] == hx.PA_ERR_ARG
        op.close()
