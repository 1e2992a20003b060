"""Benchmark: GDOF/s of the fused FP64 PA diffusion apply on one MI355X, plus the
Jacobi-PCG time to a 1e-8 relative residual, next to the CPU oracle.

Workload (one step = one operator apply y = K x, the whole fused kernel):
  48^3 hexahedra of the unit cube, interior vertices perturbed by U[-0.1h, 0.1h],
  p = 4 (GLL nodes), Q = 6 Gauss points per axis, kappa = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z),
  x ~ U[-1, 1]: 7,189,057 DOFs.  Inputs are resident in HBM before timing starts.

Prints one JSON line.  `--sweep` adds the p = 2, 4, 6, 8 mass/diffusion sweep (~30 M DOFs each).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E


# the translation unit of the apply kernels (its own sources and the build flags)
APPLY_SOURCES = ("csrc/k_apply.hip", "csrc/apply_passes.h", "csrc/apply_common.h", "csrc/internal.h",
                 "../include/hexpa.h", "build.py")


def kernel_source_hash():
    """SHA-256 over the sources the apply kernels are compiled from (traffic figures are
    tied to it)."""
    import hashlib
    h = hashlib.sha256()
    for name in APPLY_SOURCES:
        h.update(name.encode())
        with open(os.path.join(ROOT, "paper_2603_09038_amd", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(tag):
    """HBM bytes per launch from a committed rocprofv3 counter summary (profiles/<tag>.md),
    or None when the summary is absent or was taken on different kernel sources."""
    path = os.path.join(ROOT, "profiles", tag + ".md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if line.startswith("- ") and ":" in line:
                k, v = line[2:].split(":", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel source hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm bytes per launch"])
    except (KeyError, ValueError):
        return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def alg_bytes(ndof, nelem, p, q, ops):
    """Algorithmic HBM bytes of one apply: D (FP64), the int32 DOF map, read x, write y."""
    ncomp = (6 if ops & 2 else 0) + (1 if ops & 1 else 0)
    return nelem * ncomp * q ** 3 * 8 + nelem * (p + 1) ** 3 * 4 + 16 * ndof


def alg_flops(nelem, p, q, ops):
    """Sum-factorised FLOPs per element (multiply-add = 2), no MFMA padding:
    diffusion 2 [2 (2Qd^3 + 3Q^2d^2 + 3Q^3d) + 9Q^3], mass 2 [2 (Qd^3 + Q^2d^2 + Q^3d) + Q^3]."""
    d = p + 1
    f = 0
    if ops & 2:
        f += 2 * (2 * (2 * q * d ** 3 + 3 * q * q * d * d + 3 * q ** 3 * d) + 9 * q ** 3)
    if ops & 1:
        f += 2 * (2 * (q * d ** 3 + q * q * d * d + q ** 3 * d) + q ** 3)
    return nelem * f


def time_kernel(op, hexpa, x, y, steps, warmup):
    """Average duration of the fused kernel alone (pa_apply_add: one launch), HIP events on
    the stream the kernel is launched on, and the median of per-apply (fill + kernel) times."""
    import torch
    s = torch.cuda.current_stream()
    for _ in range(warmup):
        hexpa.pa_apply(op.h, x, y)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    for a, b in ev:
        a.record(s)
        hexpa.pa_apply_add(op.h, x, y)
        b.record(s)
    torch.cuda.synchronize()
    kern = [a.elapsed_time(b) for a, b in ev]
    return float(np.mean(kern)), float(np.median(kern))


def energy_per_dof(op, hexpa, x, y, ndof, seconds=3.0):
    """Throughput per watt of sustained applies (the paper's MDOF/W, Table VI): the socket
    power the driver reports, sampled every 20 ms while batches of applies run back to back
    (the first 0.5 s, while clocks and power settle, are dropped).  Returns None with the
    reason when the power readout is not available."""
    import torch
    try:
        import amdsmi
    except Exception as e:  # noqa: BLE001
        return {"error": f"amdsmi not importable: {e}"}
    try:
        amdsmi.amdsmi_init()
    except Exception as e:  # noqa: BLE001
        return {"error": f"amdsmi_init failed: {e}"}
    try:
        handles = amdsmi.amdsmi_get_processor_handles()
        h = handles[0] if len(handles) == 1 else None
        try:
            bus = torch.cuda.get_device_properties(0).pci_bus_id
            for hh in handles:
                bdf = amdsmi.amdsmi_get_gpu_device_bdf(hh)
                if int(bdf.split(":")[1], 16) == bus:
                    h = hh
        except Exception:  # noqa: BLE001
            pass
        if h is None:
            return {"error": f"cannot tell which of {len(handles)} devices runs the applies"}

        def watts():
            info = amdsmi.amdsmi_get_power_info(h)
            for key in ("current_socket_power", "average_socket_power"):
                v = info.get(key)
                if isinstance(v, (int, float)) and v > 0:
                    return float(v), key
            return None, None

        if watts()[0] is None:
            return {"error": "no socket power reading"}
        samples, key = [], None
        batch = 100

        def enqueue():
            for _ in range(batch):
                hexpa.pa_apply(op.h, x, y)
            ev = torch.cuda.Event()
            ev.record()
            return ev

        # two batches in flight, so the device never waits for the host between batches
        for _ in range(3):
            enqueue()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pending = enqueue()
        n_done, t_start, t_end = 0, None, None
        while True:
            nxt = enqueue() if time.perf_counter() - t0 < seconds else None
            while not pending.query():
                time.sleep(0.02)
                w, key = watts()
                if t_start is not None and w is not None:
                    samples.append(w)
            now = time.perf_counter()
            if t_start is None:
                if now - t0 >= 0.5:
                    t_start = now  # the batches completing after this point are counted
            else:
                n_done += batch
                t_end = now
            if nxt is None:
                break
            pending = nxt
        torch.cuda.synchronize()
        if t_start is None or not samples or n_done == 0:
            return {"error": "window too short"}
        dt = t_end - t_start
        w = float(np.mean(samples))
        rate = n_done * ndof / dt
        return {"watts_mean": w, "watts_min": float(np.min(samples)), "watts_max": float(np.max(samples)),
                "samples": len(samples), "source": f"amdsmi {key}", "applies": n_done, "seconds": dt,
                "gdofs": rate / 1e9, "mdof_per_watt": rate / 1e6 / w}
    except Exception as e:  # noqa: BLE001
        return {"error": f"{type(e).__name__}: {e}"}
    finally:
        try:
            amdsmi.amdsmi_shut_down()
        except Exception:  # noqa: BLE001
            pass


def cpu_baseline(mesh, p, q, coeff_o, ops_o, ndof, nelem, budget_s):
    import oracle
    P = oracle.Problem(mesh, p, q, coeff=coeff_o, ops=ops_o)
    x = np.random.default_rng(7).uniform(-1, 1, ndof)
    rng = np.random.default_rng(11)
    n_try = 8 * max(1, oracle.num_threads())
    P.apply(x, subset=np.sort(rng.choice(nelem, 8, replace=False)))  # warm the thread pool
    t0 = time.perf_counter()
    P.apply(x, subset=np.sort(rng.choice(nelem, n_try, replace=False)))
    t_try = time.perf_counter() - t0
    n_el = int(min(nelem, max(n_try, n_try * budget_s / max(t_try, 1e-6))))
    sub = np.sort(rng.choice(nelem, n_el, replace=False))
    t0 = time.perf_counter()
    P.apply(x, subset=sub)
    t = time.perf_counter() - t0
    dofs_equiv = ndof * n_el / nelem
    return {"value": dofs_equiv / t / 1e9, "unit": "GDOF/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{n_el} of {nelem} elements (random, seed 11), element matrices assembled on the fly "
                      f"by quadrature loops and applied; {t:.1f} s; throughput scaled by the DOF share"}


def run_cg(hexpa, mesh, coeff, p, q):
    import torch
    import synth
    op = hexpa.PAOperator(mesh, p, q, coeff=coeff, ops=hexpa.PA_DIFFUSION, ess_mode=1)
    xq = op.qpoints().cpu().numpy().reshape(-1, 3)
    b = op.load(torch.tensor(synth.f_manufactured(xq).reshape(op.nelem, -1), device="cuda"))
    ess = torch.tensor(hexpa.pa_get_ess(op.h), device="cuda", dtype=torch.long)
    b[ess] = 0.0
    torch.cuda.synchronize()
    x = torch.zeros_like(b)
    res = hexpa.cg_solve(op.h, b, x, rtol=1e-8, max_it=20000, mode=hexpa.PA_CG_JACOBI, check_every=1,
                         raise_on_fail=False)
    u = torch.tensor(synth.u_manufactured(op.nodes().cpu().numpy()), device="cuda")
    err = float((x - u).abs().max())
    op.close()
    return {"mode": "jacobi_pcg_fp64", "rtol": 1e-8, "iters": res["iters"], "seconds": res["seconds"],
            "rel_res_true": res["rel_res_true"], "status": res["rc"], "max_nodal_error_vs_exact_u": err}


RU_PERIOD = 40  # reliable-update mixed CG: most iterations between FP64 residual replacements


def run_mixed(hexpa, n=32, p=6, q=8):
    """Log-normal coefficient (sigma = 1, correlation length 0.1, draw 0), Dirichlet,
    b = A_c x* with x* the nodal interpolant of sin(pi x) sin(pi y) sin(pi z): FP64
    Jacobi-PCG against the mixed-precision solvers (refinement and FCG outer loops around
    an FP32 inner Jacobi-PCG with the FP16 / BF16 apply, and one FP32 recurrence with
    reliable updates)."""
    import torch
    import synth
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    grid, contrast = synth.lognormal_kappa_grid(0, sigma=1.0, ell=0.1)
    op = hexpa.PAOperator(mesh, p, q, coeff={"kind": hexpa.PA_COEFF_GRID, "grid": grid}, ops=hexpa.PA_DIFFUSION,
                          ess_mode=1)
    xs = torch.tensor(synth.u_manufactured(op.nodes().cpu().numpy()), device="cuda")
    b = op.apply_constrained(xs)
    out = {"workload": f"{n}^3 perturbed hex mesh, p={p}, Q={q}, log-normal kappa (contrast {contrast:.0f}), "
                       f"Dirichlet, b = A x*", "ndof": op.ndof}
    # warm the kernels (and the lazily built FP32 D)
    for fmt in (hexpa.PA_LP_FP16, hexpa.PA_LP_BF16):
        x = torch.zeros_like(b)
        hexpa.cg_solve(op.h, b, x, rtol=1e-2, max_it=1, mode=hexpa.PA_CG_MIXED_IR, lp_fmt=fmt, inner_max=5,
                       raise_on_fail=False)
    # normwise error of the 16-bit apply against the FP64 apply (unconstrained operator) for
    # a rough input (x ~ U[-1,1]) and a smooth one (the manufactured x*): rounding the
    # interpolated tile before differentiating costs more, relative to |A x|, when A x is small
    xr = torch.tensor(synth.rand_x(op.ndof, 1), device="cuda")
    lp_err = {}
    for xname, xin in (("rough", xr), ("smooth", xs)):
        ref = op.apply(xin)
        for name, fmt in (("fp16", hexpa.PA_LP_FP16), ("bf16", hexpa.PA_LP_BF16)):
            y16 = op.apply_lp(xin.float(), fmt=fmt).double()
            lp_err[f"{name}_{xname}"] = float(torch.linalg.norm(y16 - ref) / torch.linalg.norm(ref))
    out["lp_apply_rel_err"] = lp_err
    log(f"16-bit apply error vs FP64: {lp_err}")
    for tol in (1e-8, 1e-10):
        x = torch.zeros_like(b)
        r = hexpa.cg_solve(op.h, b, x, rtol=tol, max_it=50000, mode=hexpa.PA_CG_JACOBI, check_every=8,
                           raise_on_fail=False)
        err = float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs))
        out[f"fp64_pcg_{tol:.0e}"] = {"seconds": r["seconds"], "iters": r["iters"], "rel_res_true": r["rel_res_true"],
                                      "rel_err_vs_xstar": err, "status": r["rc"]}
        # outer FP64 iterative refinement (inner tolerance 1e-1) and FP64 FCG outer (3e-2):
        # the settings that were fastest for each in a sweep of 0.3 ... 1e-4
        for outer, mode, itol in (("ir", hexpa.PA_CG_MIXED_IR, 1e-1), ("fcg", hexpa.PA_CG_MIXED_FCG, 3e-2)):
            for name, fmt in (("fp16", hexpa.PA_LP_FP16), ("bf16", hexpa.PA_LP_BF16)):
                x = torch.zeros_like(b)
                r = hexpa.cg_solve(op.h, b, x, rtol=tol, max_it=200, mode=mode, lp_fmt=fmt, inner_rtol=itol,
                                   inner_max=3000, check_every=8, raise_on_fail=False)
                err = float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs))
                key = f"mixed_{outer}_{name}_{tol:.0e}"
                out[key] = {"seconds": r["seconds"], "outer": r["iters"], "inner_iters": r["inner_iters_total"],
                            "inner_rtol": itol, "rel_res_true": r["rel_res_true"], "rel_err_vs_xstar": err,
                            "status": r["rc"]}
                out[f"speedup_{outer}_{name}_{tol:.0e}"] = out[f"fp64_pcg_{tol:.0e}"]["seconds"] / r["seconds"]
        # one FP32 recurrence with reliable updates (FP64 residual replacement at most every
        # RU_PERIOD iterations), with the FP16 apply and with the BF16 apply (whose element
        # tiles are centred on their means before rounding)
        for name, fmt in (("fp16", hexpa.PA_LP_FP16), ("bf16", hexpa.PA_LP_BF16)):
            x = torch.zeros_like(b)
            r = hexpa.cg_solve(op.h, b, x, rtol=tol, max_it=20000, mode=hexpa.PA_CG_MIXED_RU, lp_fmt=fmt,
                               inner_max=RU_PERIOD, raise_on_fail=False)
            err = float(torch.linalg.norm(x - xs) / torch.linalg.norm(xs))
            out[f"mixed_ru_{name}_{tol:.0e}"] = {"seconds": r["seconds"], "replacements": r["iters"],
                                                 "iters": r["inner_iters_total"], "period_max": RU_PERIOD,
                                                 "rel_res_true": r["rel_res_true"], "rel_err_vs_xstar": err,
                                                 "status": r["rc"]}
            out[f"speedup_ru_{name}_{tol:.0e}"] = out[f"fp64_pcg_{tol:.0e}"]["seconds"] / r["seconds"]
    op.close()
    return out


def run_learned(hexpa, ntrain, nheld, n=32, p=4, weights=None):
    """Learned two-level preconditioner: train on log-normal draws 0..ntrain-1 (iterates of
    Jacobi-PCG on b = A_c x*_d), then on held-out draws 200.. compare FP64 Jacobi-PCG,
    FCG with coarse correction + Jacobi ("without the network") and FCG with coarse
    correction + network, each to 1e-8 from x = 0."""
    import synth
    from paper_2603_09038_amd import learned
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    op0 = learned.lognormal_operator(mesh, n, p, 0)
    lp = hexpa.LearnedPreconditioner(op0, use_net=True, use_coarse=True, coarse_iters=4, lr=1e-3)
    out = {"workload": f"{n}^3 perturbed hex mesh, p={p}, Q={p + 2}, log-normal kappa draws, Dirichlet",
           "ndof": op0.ndof, "train_draws": ntrain, "held_out_draws": nheld}
    if weights and os.path.exists(weights):
        lp.load(weights)
        out["weights"] = "loaded"
    else:
        losses, tc, tt = learned.train(lp, mesh, n, p, list(range(ntrain)), log=log)
        out.update({"train_steps": len(losses), "train_seconds": tt, "capture_seconds": tc,
                    "loss_first": float(np.mean(losses[:16])), "loss_last": float(np.mean(losses[-16:]))})
    rows = learned.compare(lp, mesh, n, p, list(range(200, 200 + nheld)), log=log)
    for key in ("jacobi", "coarse_jacobi", "coarse_net"):
        out[key] = {"iters": [r[key]["iters"] for r in rows], "seconds": [r[key]["seconds"] for r in rows],
                    "rel_res_true": [r[key]["rel_res_true"] for r in rows],
                    "status": [r[key]["rc"] for r in rows]}
        out[key]["seconds_mean"] = float(np.mean(out[key]["seconds"]))
        out[key]["iters_mean"] = float(np.mean(out[key]["iters"]))
    out["fallbacks"] = sum(r["coarse_net"]["fallback"] for r in rows)
    out["contrast"] = [r["contrast"] for r in rows]
    out["speedup_net_vs_jacobi"] = out["jacobi"]["seconds_mean"] / out["coarse_net"]["seconds_mean"]
    out["speedup_net_vs_coarse_jacobi"] = out["coarse_jacobi"]["seconds_mean"] / out["coarse_net"]["seconds_mean"]
    lp.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    # 200 untimed applies (~70 ms) let the clocks reach their sustained level first
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--variant", default="auto", choices=["auto", "mfma", "valu", "colored"])
    ap.add_argument("--cpu-budget", type=float, default=15.0, help="seconds of oracle CPU work (0 = skip)")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-matrix", action="store_true", help="skip the unfused/fused/matrix-free kernel matrix")
    ap.add_argument("--no-energy", action="store_true", help="skip the MDOF/W measurement")
    ap.add_argument("--learned-train", type=int, default=40, help="training draws of the learned preconditioner")
    ap.add_argument("--learned-held", type=int, default=20, help="held-out draws of the learned comparison")
    ap.add_argument("--learned-weights", default=None, help="load parameters from this file instead of training")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (for HBM counter calibration)")
    ap.add_argument("--sweep", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2603_09038_amd import hexpa
    torch.cuda.set_device(0)
    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.float64, device="cuda")
        c = torch.empty_like(a)
        for _ in range(3):
            c.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 8, "copy_bytes_written": a.numel() * 8}), flush=True)
        return

    n, p, q = 48, 4, 6
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    coeff = {"kind": hexpa.PA_COEFF_SINE, "value": 1.0, "amp": 0.5, "freq": 2.0}
    op = hexpa.PAOperator(mesh, p, q, coeff=coeff, ops=hexpa.PA_DIFFUSION)
    VAR = {"mfma": hexpa.PA_VARIANT_MFMA, "valu": hexpa.PA_VARIANT_VALU, "colored": hexpa.PA_VARIANT_MFMA_COLORED}
    VNAME = {v: k for k, v in VAR.items()}
    if args.variant != "auto":
        op.set_variant(VAR[args.variant])
    used = VNAME[op.info["variant"]]
    ndof, nelem = op.ndof, op.nelem
    x = torch.tensor(synth.rand_x(ndof, 0), device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()

    # timed region: exactly `steps` full applies (fill + fused kernel)
    for _ in range(args.warmup):
        hexpa.pa_apply(op.h, x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        hexpa.pa_apply(op.h, x, y)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = 1e3 * wall / args.steps
    gdofs = ndof / (wall / args.steps) / 1e9

    log(f"timed {args.steps} applies: {ms_step:.4f} ms/step")
    k_mean_ms, k_med_ms = time_kernel(op, hexpa, x, y, args.steps, 3)
    ab = alg_bytes(ndof, nelem, p, q, 2)
    achieved = ab / (k_mean_ms * 1e-3) / 1e9
    out = {
        "metric": "GDOF/s PA diffusion apply p=2..8; CG time-to-1e-8 mixed/learned vs FP64",
        "value": gdofs, "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "fp64 PA diffusion apply, 48^3 perturbed hex mesh, p=4, Q=6, "
                               "kappa=1+0.5sin(2pi x)sin(2pi y)sin(2pi z), x~U[-1,1]",
                   "ndof": ndof, "nelem": nelem, "p": p, "q1d": q, "variant": used},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(f"k_apply_c2_p4_diffusion_{used}_hbm_traffic"),
                     "kernel": f"k_apply<D=5,Q=6,diffusion,{used}>", "alg_bytes_per_launch": ab,
                     "alg_bytes_per_dof": ab / ndof, "kernel_ms_mean": k_mean_ms, "kernel_ms_median": k_med_ms,
                     "kernel_gdofs": ndof / (k_mean_ms * 1e-3) / 1e9,
                     "fp64_frac": alg_flops(nelem, p, q, 2) / (k_mean_ms * 1e-3) / 78.6e12},
    }
    # the paper's kernel matrix at this workload: {unfused PA, fused PA, fused matrix-free} x
    # {vector ALU, MFMA}; the unfused apply moves the quadrature-point tensor through HBM four
    # more times, the matrix-free one reads no D (vertex coordinates instead)
    qt_bytes = 8 * 3 * q ** 3 * nelem
    matrix = []
    mf_bytes = ab - 8 * 6 * q ** 3 * nelem + nelem * (8 * 4 + 24 * 8)  # no D; hex indices + vertex coordinates
    variants = (("fused_valu", hexpa.PA_VARIANT_VALU), ("fused_mfma", hexpa.PA_VARIANT_MFMA),
                ("unfused_valu", hexpa.PA_VARIANT_VALU_UNFUSED), ("unfused_mfma", hexpa.PA_VARIANT_MFMA_UNFUSED),
                ("fused_mf_valu", hexpa.PA_VARIANT_VALU_MF), ("fused_mf_mfma", hexpa.PA_VARIANT_MFMA_MF))
    for name, v in (() if args.no_matrix else variants):
        op.set_variant(v)
        km, _ = time_kernel(op, hexpa, x, y, 30, 10)
        hb = ab + 4 * qt_bytes if name.startswith("unfused") else (mf_bytes if "_mf_" in name else ab)
        matrix.append({"variant": name, "ms": km, "gdofs": ndof / (km * 1e-3) / 1e9, "hbm_bytes_model": hb,
                       "hbm_frac_model": hb / (km * 1e-3) / 1e9 / HBM_PEAK_GBS})
        log(f"kernel matrix {name}: {km:.4f} ms")
    op.set_variant(VAR[used])
    if matrix:
        out["kernel_matrix"] = matrix
    if not args.no_energy:
        out["energy"] = energy_per_dof(op, hexpa, x, y, ndof)
        log(f"energy: {out['energy']}")
    if not args.no_cg:
        out["cg"] = run_cg(hexpa, mesh, coeff, p, q)
        log(f"C2 Jacobi-PCG: {out['cg']['iters']} iterations, {out['cg']['seconds']:.3f} s")
    op.close()
    if not args.no_mixed:
        out["mixed"] = run_mixed(hexpa)
        log("mixed-precision comparison done")
    if not args.no_learned:
        out["learned"] = run_learned(hexpa, args.learned_train, args.learned_held, weights=args.learned_weights)
        log("learned-preconditioner comparison done")
    if args.sweep:
        sweep = []
        for pp, nn in ((2, 155), (4, 78), (6, 52), (8, 40)):
            m2 = synth.box_mesh(nn, perturb=0.1, seed=0)
            for ops in (hexpa.PA_MASS, hexpa.PA_DIFFUSION):
                o2 = hexpa.PAOperator(m2, pp, pp + 2, ops=ops)
                if args.variant != "auto":
                    o2.set_variant(VAR[args.variant])
                x2 = torch.tensor(synth.rand_x(o2.ndof, 0), device="cuda")
                y2 = torch.empty_like(x2)
                km, _ = time_kernel(o2, hexpa, x2, y2, 20, 5)
                ab2 = alg_bytes(o2.ndof, o2.nelem, pp, pp + 2, ops)
                sweep.append({"p": pp, "n": nn, "op": "mass" if ops == 1 else "diffusion", "ndof": o2.ndof,
                              "kernel_ms": km, "gdofs": o2.ndof / (km * 1e-3) / 1e9,
                              "hbm_frac": ab2 / (km * 1e-3) / 1e9 / HBM_PEAK_GBS,
                              "variant": VNAME[o2.info["variant"]]})
                log(f"sweep p={pp} ops={ops}: {sweep[-1]['gdofs']:.2f} GDOF/s")
                o2.close()
                del x2, y2
                torch.cuda.empty_cache()
        out["sweep"] = sweep
    if args.cpu_budget > 0:
        import oracle
        log("CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(mesh, p, q, oracle.Coeff.sine(), oracle.DIFFUSION, ndof, nelem,
                                           args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
