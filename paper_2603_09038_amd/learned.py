"""Training and evaluation of the learned two-level preconditioner (orchestration only).

Every numerical step runs in the library: the Jacobi-PCG that produces the training
iterates (cg_solve with iterate capture), the residuals and targets, the network's
forward and backward passes and Adam (pa_lp_train_step), and the FCG solves that compare
the preconditioners.  This module only chooses coefficient draws, builds operators and
loops over them.

Training data (per draw d): the system A_c x = b_c with a known solution x*_d, b_c =
A_c x*_d, solved by FP64 Jacobi-PCG from 0; the iterates x_k at roughly log-spaced k give
pairs (r_k = b_c - A_c x_k, e_k = x*_d - x_k) with the exact error known without a tight
solve.  The network part is trained on the target e_k minus the coarse correction of r_k.
"""
import time

import numpy as np

from . import hexpa

# roughly log-spaced iteration numbers, 0 = the first residual b: for Jacobi-PCG
# (Fibonacci-like, up to ~1600) and for FCG with the two-level preconditioner (~150)
CAPTURE_AT = (0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233, 377, 610, 987, 1597)
CAPTURE_AT_FCG = (0, 1, 2, 3, 4, 6, 8, 11, 15, 20, 27, 36, 48, 64, 85, 113, 150)


def lognormal_operator(mesh, n, p, draw, sigma=1.0, ell=0.1, nfft=128):
    # nfft: FFT grid of the random field over [0, 2)^3 (128 for the workloads; 64 is a
    # cheaper field with the same correlation length for tests)
    """PA diffusion operator (Q = p + 2, Dirichlet box boundary) with kappa = exp(sigma g_draw)."""
    import synth
    grid, contrast = synth.lognormal_kappa_grid(draw, sigma=sigma, ell=ell, nfft=nfft)
    op = hexpa.PAOperator(mesh, p, p + 2, coeff={"kind": hexpa.PA_COEFF_GRID, "grid": grid},
                          ops=hexpa.PA_DIFFUSION, ess_mode=1)
    op.contrast = contrast
    return op


def capture_iterates(op, xstar, lp=None, max_it=None, capture_at=None):
    """b = A_c x*, and the iterates x_k at the listed k that the solve reaches: Jacobi-PCG
    (lp None) or FCG preconditioned by lp as it is configured (the distribution of
    residuals the network meets in use)."""
    import torch
    b = op.apply_constrained(xstar)
    if capture_at is None:
        capture_at = CAPTURE_AT if lp is None else CAPTURE_AT_FCG
    if max_it is None:
        max_it = capture_at[-1] + 1
    cap = torch.empty((len(capture_at), op.ndof), dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    mode = hexpa.PA_CG_JACOBI if lp is None else hexpa.PA_CG_FCG
    res = hexpa.cg_solve(op.h, b, x, rtol=1e-10, max_it=max_it, mode=mode, capture_at=capture_at, capture_x=cap,
                         check_every=8, lp=None if lp is None else lp.h, raise_on_fail=False)
    reached = [j for j, k in enumerate(capture_at) if k <= res["iters"]]
    return b, cap[reached], res


def train(lp, mesh, n, p, draws, epochs=1, seed=0, sigma=1.0, log=None, capture="fcg", nfft=128, chunk=50):
    """Train lp's network on the iterates of the given coefficient draws: the library's
    pa_lp_train runs the capture solves (FCG with the preconditioner as it currently is,
    capture "fcg" -- the untrained network adds nothing, so the first pass sees the
    two-level method without it -- or Jacobi-PCG, "jacobi") and the training steps.  This
    function only builds the operators of `chunk` draws at a time (bounding device
    memory) and hands them over.  Returns per-step losses and the seconds spent (building
    the operators and capturing; training)."""
    import synth
    import torch
    losses, t_capture, t_train = [], 0.0, 0.0
    at = CAPTURE_AT_FCG if capture == "fcg" else CAPTURE_AT
    mode = hexpa.PA_LP_CAPTURE_FCG if capture == "fcg" else hexpa.PA_LP_CAPTURE_JACOBI
    for ep in range(epochs):
        for c0 in range(0, len(draws), chunk):
            t0 = time.perf_counter()
            ops, xs = [], []
            for d in draws[c0:c0 + chunk]:
                op = lognormal_operator(mesh, n, p, d, sigma=sigma, nfft=nfft)
                ops.append(op)
                xs.append(torch.tensor(synth.train_solution(op.nodes().cpu().numpy(), d), dtype=torch.float64,
                                       device="cuda"))
            torch.cuda.synchronize()
            t_build = time.perf_counter() - t0
            ls, tc, tt = lp.train(ops, xs, at, capture=mode, epochs=1, seed=seed * 1000003 + ep * 1009 + c0)
            losses.extend(ls.tolist())
            t_capture += t_build + tc
            t_train += tt
            if log:
                log(f"epoch {ep} draws {draws[c0]}..{draws[min(c0 + chunk, len(draws)) - 1]}: {len(ls)} steps, "
                    f"mean loss {np.mean(ls):.4f}")
            del xs
            for op in ops[:-1]:  # lp keeps the last one, to which the handle stays bound
                op.close()
    return losses, t_capture, t_train


def compare(lp, mesh, n, p, draws, rtol=1e-8, sigma=1.0, coarse_iters=None, max_it=20000, log=None, net_scale=1.0,
            nfft=128):
    """Iterations and seconds to rtol on held-out draws for (i) Jacobi-PCG, (ii) FCG with
    Jacobi + coarse correction (the preconditioner without the network), (iii) FCG with
    network + coarse correction.  The right-hand side is b = A_c x* with x* the nodal
    interpolant of sin(pi x) sin(pi y) sin(pi z)."""
    import synth
    import torch
    rows = []
    for d in draws:
        op = lognormal_operator(mesh, n, p, d, sigma=sigma, nfft=nfft)
        xstar = torch.tensor(synth.u_manufactured(op.nodes().cpu().numpy()), dtype=torch.float64, device="cuda")
        b = op.apply_constrained(xstar)
        lp.bind(op)
        row = {"draw": d, "contrast": op.contrast}
        x = torch.zeros_like(b)
        row["jacobi"] = hexpa.cg_solve(op.h, b, x, rtol=rtol, max_it=max_it, mode=hexpa.PA_CG_JACOBI,
                                       check_every=8, raise_on_fail=False)
        for key, use_net in (("coarse_jacobi", False), ("coarse_net", True)):
            kw = {} if coarse_iters is None else {"coarse_iters": coarse_iters}
            lp.configure(use_net=use_net, use_coarse=True, net_scale=net_scale, **kw)
            x = torch.zeros_like(b)
            row[key] = hexpa.cg_solve(op.h, b, x, rtol=rtol, max_it=max_it, mode=hexpa.PA_CG_FCG, lp=lp.h,
                                      check_every=4, raise_on_fail=False)
        rows.append(row)
        if log:
            log("draw %d: jacobi %d it %.3fs | fcg coarse+jacobi %d it %.3fs | fcg coarse+net %d it %.3fs%s" % (
                d, row["jacobi"]["iters"], row["jacobi"]["seconds"], row["coarse_jacobi"]["iters"],
                row["coarse_jacobi"]["seconds"], row["coarse_net"]["iters"], row["coarse_net"]["seconds"],
                " (fallback)" if row["coarse_net"]["fallback"] else ""))
    return rows
