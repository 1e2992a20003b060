"""Seeded synthetic inputs shared by the HIP path's tests/bench and by the CPU oracle.

This module produces *inputs only*: hexahedral box meshes (vertex coordinates and
corner connectivity), random vectors, coefficient grids and pointwise analytic
functions.  It holds none of the finite-element arithmetic (no basis functions,
no quadrature, no geometric factors, no operator action), so neither side of a
parity comparison can borrow the other's method through it.

Random streams use numpy's PCG64 seeded as ``default_rng([seed, stream])`` with
stream 0 = mesh perturbation, 1 = input vector, 2 = coefficient field,
3 = auxiliary field for training right-hand sides, 7 = network parameters.
"""
from .fixtures import (  # noqa: F401
    box_mesh,
    affine_box_mesh,
    rand_x,
    grf_grid,
    lognormal_kappa_grid,
    sine_kappa,
    u_manufactured,
    f_manufactured,
    trilinear_sample,
    net_params,
    flat_params,
    train_solution,
    STREAM_MESH,
    STREAM_X,
    STREAM_FIELD,
    STREAM_AUX,
)
