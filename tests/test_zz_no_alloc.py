"""pa_apply_unfused_noalloc (the unfused apply with its quadrature-point tensor in the
library's fixed device array) against pa_apply with the same unfused variant, which
stages the tensor in handle memory: two calls in a row, the second on a smaller operator,
each within the FP64 parity bar (1e-12 normwise, 2-norm and max-norm; the atomic scatter
makes the summation order differ between launches), and the size limit enforced before
any launch."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

TOL = 1e-12


@pytest.fixture(scope="module")
def hx():
    import torch  # noqa: F401
    from paper_2603_09038_amd import hexpa
    return hexpa


def _rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return max(np.linalg.norm(a - b) / np.linalg.norm(b), np.abs(a - b).max() / np.abs(b).max())


@pytest.mark.parametrize("variant_name", ["PA_VARIANT_MFMA_UNFUSED", "PA_VARIANT_VALU_UNFUSED"])
def test_noalloc_matches_unfused_apply(hx, variant_name):
    import torch
    variant = getattr(hx, variant_name)
    coeff = {"kind": hx.PA_COEFF_SINE, "value": 1.0, "amp": 0.5, "freq": 2.0}
    # first a larger operator, then a smaller one: the second call reuses the array the
    # first one filled
    for n, p, ops in ((6, 4, 3), (3, 3, 2)):
        mesh = synth.box_mesh(n, perturb=0.1, seed=40 + n)
        op = hx.PAOperator(mesh, p, p + 2, coeff=coeff, ops=ops)
        x = torch.tensor(synth.rand_x(op.ndof, n), dtype=torch.float64, device="cuda")
        y = torch.full_like(x, float("nan"))
        hx.pa_apply_unfused_noalloc(op.h, variant, x, y)
        op.set_variant(variant)
        ref = op.apply(x).cpu().numpy()
        got = y.cpu().numpy()
        assert np.all(np.isfinite(got))
        assert _rel(got, ref) <= TOL, (n, p, ops, _rel(got, ref))
        op.close()


def test_noalloc_rejects_an_operator_beyond_the_array(hx):
    import torch
    mesh = synth.box_mesh(30)  # 27,000 elements x 3 channels x 6^3 points > 16 Mi doubles
    op = hx.PAOperator(mesh, 4, 6, ops=2)
    x = torch.zeros(op.ndof, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(hx.HexpaError) as ei:
        hx.pa_apply_unfused_noalloc(op.h, hx.PA_VARIANT_MFMA_UNFUSED, x, y)
    assert ei.value.code == hx.PA_ERR_ARG
    with pytest.raises(hx.HexpaError) as ei:
        hx.pa_apply_unfused_noalloc(op.h, hx.PA_VARIANT_MFMA, x, y)
    assert ei.value.code == hx.PA_ERR_ARG
    op.close()
