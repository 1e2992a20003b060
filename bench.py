"""Benchmark of the PA operator library on one MI355X, next to the CPU oracle.

Headline (one step = one fused FP64 diffusion apply y = K x at each of p = 2, 4, 6, 8):
  the order sweep on the unit cube, Q = p + 2 Gauss points per axis, kappa = 1,
  x ~ U[-1, 1], interior vertices perturbed by U[-0.1h, 0.1h]; meshes sized to about
  30 M DOFs: p=2 on 155^3 (30,080,231 DOFs), p=4 on 78^3 (30,664,297), p=6 on 52^3
  (30,664,297), p=8 on 40^3 (33,076,161).  Inputs and operators are resident in HBM
  before timing starts.  value = (sum of the four DOF counts) x steps / wall time: the
  whole-job apply throughput over the four orders.  Every order's kernel is also timed
  with HIP events on its launch stream inside the timed region (per-order GDOF/s and
  fraction of the 8 TB/s HBM roof), and the mass operator at the same sizes afterwards.

Further legs (each can be switched off): the paper's own operator (the fused kernel of the
off-diagonal blocks of the acoustic operator, H1 p=4 x L2 p=3, Q1D=5, and its RK4 step);
the 48^3 p=4 sine-coefficient operator (kernel
roofline, the unfused / fused / matrix-free x vector-ALU / MFMA kernel matrix, MDOF/W,
Jacobi-PCG to 1e-8 with its per-iteration roofline fraction); mixed precision on the
32^3 p=6 log-normal workload; the learned preconditioner on the 32^3 p=4 log-normal
draws (200 training draws, 20 held out); the CPU oracle (element-matrix assembly and
apply timed separately on element samples, and its Jacobi-PCG on a reduced mesh).

Prints one JSON line on stdout; progress goes to stderr.
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

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6   # MI355X dense FP64 (vector and MFMA alike)
METRIC = "GDOF/s PA diffusion apply p=2..8; CG time-to-1e-8 mixed/learned vs FP64"
SWEEP = ((2, 155), (4, 78), (6, 52), (8, 40))  # (p, n): about 30 M DOFs each
CG_VEC_BYTES_PER_DOF = 112  # FP64 PCG vector kernels per iteration: p.Ap 16, x/r update 56, p update 40

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


def roof_row(ndof, nelem, p, q, ops, kernel_ms):
    ab = alg_bytes(ndof, nelem, p, q, ops)
    t = kernel_ms * 1e-3
    return {"kernel_ms": kernel_ms, "gdofs": ndof / t / 1e9, "alg_bytes": ab, "alg_bytes_per_dof": ab / ndof,
            "hbm_frac": ab / t / 1e9 / HBM_PEAK_GBS, "fp64_frac": alg_flops(nelem, p, q, ops) / t / 1e12 / FP64_PEAK_TFLOPS}


def warm(fn, seconds, min_calls=1):
    """Call fn() until `seconds` have passed (and at least min_calls times): the clocks
    reach their sustained level before anything is timed."""
    import torch
    t0 = time.perf_counter()
    k = 0
    while k < min_calls or time.perf_counter() - t0 < seconds:
        fn()
        k += 1
        if k % 20 == 0:
            torch.cuda.synchronize()
    torch.cuda.synchronize()
    return k


def stream_read_gbps(nbytes=1 << 31, launches=10):
    """Rate of a plain device-wide read on this machine: torch.sum over 2 GiB of FP64, timed
    with HIP events.  Context for the roofline fraction (the practical ceiling of a streaming
    kernel differs from machine to machine), never part of `value`."""
    import torch
    a = torch.rand(nbytes // 8, dtype=torch.float64, device="cuda")
    s = torch.cuda.current_stream()
    for _ in range(3):
        a.sum()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(launches):
        a.sum()
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / launches
    del a
    torch.cuda.empty_cache()
    return nbytes / (ms * 1e-3) / 1e9


def time_kernel(op, hexpa, x, y, launches, warm_s=0.3):
    """Mean duration of the fused kernel alone (pa_apply_add: one launch), HIP events on the
    stream the kernel is launched on (torch's current stream, which the binding passes)."""
    import torch
    s = torch.cuda.current_stream()
    warm(lambda: hexpa.pa_apply(op.h, x, y), warm_s, 3)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(launches)]
    for a, b in ev:
        a.record(s)
        hexpa.pa_apply_add(op.h, x, y)
        b.record(s)
    torch.cuda.synchronize()
    return float(np.mean([a.elapsed_time(b) for a, b in ev]))


def run_headline(hexpa, steps, warmup, warm_s, orders):
    """The timed region: `steps` passes over the diffusion operators of the order sweep."""
    import torch
    import synth
    cases = []
    for p, n in orders:
        t0 = time.perf_counter()
        mesh = synth.box_mesh(n, perturb=0.1, seed=0)
        op = hexpa.PAOperator(mesh, p, p + 2, ops=hexpa.PA_DIFFUSION)
        x = torch.tensor(synth.rand_x(op.ndof, 0), device="cuda")
        y = torch.empty_like(x)
        cases.append({"p": p, "n": n, "op": op, "x": x, "y": y})
        log(f"set up p={p} on {n}^3 ({op.ndof} DOFs) in {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()

    def one_step(events=None):
        for j, c in enumerate(cases):
            c["y"].zero_()  # y = A x: zero y, then the fused kernel adds A x
            if events is not None:
                events[j][0].record(s)
            hexpa.pa_apply_add(c["op"].h, c["x"], c["y"])
            if events is not None:
                events[j][1].record(s)

    for _ in range(warmup):
        one_step()
    warm(one_step, warm_s)
    ev = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in cases]
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        one_step(ev[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    rows = []
    VN = {hexpa.PA_VARIANT_MFMA: "mfma", hexpa.PA_VARIANT_VALU: "valu"}
    for j, c in enumerate(cases):
        op = c["op"]
        km = float(np.mean([ev[k][j][0].elapsed_time(ev[k][j][1]) for k in range(steps)]))
        r = {"p": c["p"], "q1d": c["p"] + 2, "n": c["n"], "op": "diffusion", "ndof": op.ndof, "nelem": op.nelem,
             "variant": VN.get(op.info["variant"], str(op.info["variant"])),
             "elems_per_group": op.info["elems_per_block"], "threads": op.info["threads_per_block"]}
        r.update(roof_row(op.ndof, op.nelem, c["p"], c["p"] + 2, 2, km))
        rows.append(r)
        log(f"p={c['p']} diffusion: kernel {km:.4f} ms = {r['gdofs']:.2f} GDOF/s, {100 * r['hbm_frac']:.1f} % of HBM roof")
    total = sum(c["op"].ndof for c in cases)
    for c in cases:
        c["op"].close()
    del cases
    torch.cuda.empty_cache()
    return wall, total, rows


def run_mass_sweep(hexpa, orders, launches=20):
    import torch
    import synth
    rows = []
    VN = {hexpa.PA_VARIANT_MFMA: "mfma", hexpa.PA_VARIANT_VALU: "valu"}
    for p, n in orders:
        mesh = synth.box_mesh(n, perturb=0.1, seed=0)
        op = hexpa.PAOperator(mesh, p, p + 2, ops=hexpa.PA_MASS)
        x = torch.tensor(synth.rand_x(op.ndof, 0), device="cuda")
        y = torch.empty_like(x)
        km = time_kernel(op, hexpa, x, y, launches)
        r = {"p": p, "q1d": p + 2, "n": n, "op": "mass", "ndof": op.ndof, "nelem": op.nelem,
             "variant": VN.get(op.info["variant"], str(op.info["variant"])),
             "elems_per_group": op.info["elems_per_block"], "threads": op.info["threads_per_block"]}
        r.update(roof_row(op.ndof, op.nelem, p, p + 2, 1, km))
        rows.append(r)
        log(f"p={p} mass: kernel {km:.4f} ms = {r['gdofs']:.2f} GDOF/s, {100 * r['hbm_frac']:.1f} % of HBM roof")
        op.close()
        del x, y
        torch.cuda.empty_cache()
    return rows


def energy_per_dof(op, hexpa, x, y, ndof, seconds=2.0):
    """Throughput per watt of sustained applies (the paper's MDOF/W, Table VI): the socket
    power the driver reports, sampled every 20 ms while batches of applies run back to back
    (the first 0.5 s, while clocks and power settle, are dropped).  Returns the reason when
    the power readout is not available."""
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


def c2_problem(hexpa, n=48, p=4, q=6):
    """48^3 perturbed mesh, p=4, Q=6, kappa = 1 + 0.5 sin(2 pi x) sin(2 pi y) sin(2 pi z)."""
    import synth
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    coeff = {"kind": hexpa.PA_COEFF_SINE, "value": 1.0, "amp": 0.5, "freq": 2.0}
    return mesh, coeff


def gpu_cg(hexpa, mesh, coeff, p, q, check_every=1):
    """Jacobi-PCG to 1e-8 on the manufactured right-hand side with Dirichlet conditions."""
    import torch
    import synth
    op = hexpa.PAOperator(mesh, p, q, coeff=coeff, ops=hexpa.PA_DIFFUSION, ess_mode=1)
    xq = op.qpoints().cpu().numpy().reshape(-1, 3)
    b = op.load(torch.tensor(synth.f_manufactured(xq).reshape(op.nelem, -1), device="cuda"))
    ess = torch.tensor(hexpa.pa_get_ess(op.h), device="cuda", dtype=torch.long)
    b[ess] = 0.0
    x = torch.zeros_like(b)
    hexpa.cg_solve(op.h, b, x, rtol=1e-2, max_it=50, mode=hexpa.PA_CG_JACOBI, raise_on_fail=False)  # warm
    x.zero_()
    torch.cuda.synchronize()
    res = hexpa.cg_solve(op.h, b, x, rtol=1e-8, max_it=20000, mode=hexpa.PA_CG_JACOBI, check_every=check_every,
                         raise_on_fail=False)
    u = torch.tensor(synth.u_manufactured(op.nodes().cpu().numpy()), device="cuda")
    err = float((x - u).abs().max())
    out = {"ndof": op.ndof, "iters": res["iters"], "seconds": res["seconds"], "rel_res_true": res["rel_res_true"],
           "status": res["rc"], "max_nodal_error_vs_exact_u": err}
    op.close()
    return out


def run_c2(hexpa, args):
    """The 48^3 p=4 workload: kernel roofline, kernel matrix, MDOF/W, diag cost, Jacobi-PCG."""
    import torch
    import synth
    n, p, q = 48, 4, 6
    mesh, coeff = c2_problem(hexpa)
    op = hexpa.PAOperator(mesh, p, q, coeff=coeff, ops=hexpa.PA_DIFFUSION)
    x = torch.tensor(synth.rand_x(op.ndof, 0), device="cuda")
    y = torch.empty_like(x)
    VN = {hexpa.PA_VARIANT_MFMA: "mfma", hexpa.PA_VARIANT_VALU: "valu"}
    used = VN[op.info["variant"]]
    km = time_kernel(op, hexpa, x, y, 50)
    out = {"workload": "fp64 PA diffusion apply, 48^3 perturbed hex mesh, p=4, Q=6, "
                       "kappa=1+0.5sin(2pi x)sin(2pi y)sin(2pi z), x~U[-1,1]",
           "ndof": op.ndof, "nelem": op.nelem, "variant": used}
    out.update(roof_row(op.ndof, op.nelem, p, q, 2, km))
    out["traffic"] = measured_traffic(f"k_apply_c2_p4_diffusion_{used}_hbm_traffic")
    log(f"C2 kernel {km:.4f} ms = {out['gdofs']:.2f} GDOF/s, {100 * out['hbm_frac']:.1f} % of HBM roof")
    # diag against applies
    d = torch.empty_like(x)
    hexpa.pa_diag(op.h, d)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(10):
        hexpa.pa_diag(op.h, d)
    e1.record(s)
    torch.cuda.synchronize()
    out["diag_ms"] = e0.elapsed_time(e1) / 10
    out["diag_in_applies"] = out["diag_ms"] / km
    if not args.no_matrix:
        # the paper's kernel matrix: {unfused PA, fused PA, fused matrix-free} x {vector ALU,
        # MFMA}; the unfused apply moves the quadrature-point tensor through HBM four more
        # times, the matrix-free one reads vertex coordinates instead of D
        ab = alg_bytes(op.ndof, op.nelem, p, q, 2)
        qt_bytes = 8 * 3 * q ** 3 * op.nelem
        mf_bytes = ab - 8 * 6 * q ** 3 * op.nelem + op.nelem * (8 * 4 + 24 * 8)
        matrix = []
        for name, v in (("fused_valu", hexpa.PA_VARIANT_VALU), ("fused_mfma", hexpa.PA_VARIANT_MFMA),
                        ("unfused_valu", hexpa.PA_VARIANT_VALU_UNFUSED), ("unfused_mfma", hexpa.PA_VARIANT_MFMA_UNFUSED),
                        ("fused_mf_valu", hexpa.PA_VARIANT_VALU_MF), ("fused_mf_mfma", hexpa.PA_VARIANT_MFMA_MF)):
            op.set_variant(v)
            kmv = time_kernel(op, hexpa, x, y, 30, 0.1)
            hb = ab + 4 * qt_bytes if name.startswith("unfused") else (mf_bytes if "_mf_" in name else ab)
            matrix.append({"variant": name, "ms": kmv, "gdofs": op.ndof / (kmv * 1e-3) / 1e9, "hbm_bytes_model": hb,
                           "hbm_frac_model": hb / (kmv * 1e-3) / 1e9 / HBM_PEAK_GBS})
            log(f"kernel matrix {name}: {kmv:.4f} ms")
        op.set_variant(hexpa.PA_VARIANT_VALU if used == "valu" else hexpa.PA_VARIANT_MFMA)
        out["kernel_matrix"] = matrix
    if not args.no_energy:
        out["energy"] = energy_per_dof(op, hexpa, x, y, op.ndof)
        log(f"energy: {out['energy']}")
    apply_bytes = alg_bytes(op.ndof, op.nelem, p, q, 2)
    op.close()
    del x, y, d
    if not args.no_cg:
        cg = gpu_cg(hexpa, mesh, coeff, p, q)
        it_s = cg["seconds"] / max(cg["iters"], 1)
        it_bytes = apply_bytes + CG_VEC_BYTES_PER_DOF * cg["ndof"]
        cg.update({"mode": "jacobi_pcg_fp64", "rtol": 1e-8, "ms_per_iter": 1e3 * it_s,
                   "alg_bytes_per_iter": it_bytes, "hbm_frac_per_iter": it_bytes / it_s / 1e9 / HBM_PEAK_GBS})
        log(f"C2 Jacobi-PCG: {cg['iters']} iterations, {cg['seconds']:.3f} s, "
            f"{100 * cg['hbm_frac_per_iter']:.1f} % of HBM roof per iteration")
        # the same solve on a reduced mesh, for the oracle's PCG beside it
        red = gpu_cg(hexpa, synth.box_mesh(args.cg_reduced_n, perturb=0.1, seed=0), coeff, p, q)
        red["mesh"] = f"{args.cg_reduced_n}^3"
        cg["reduced_mesh_gpu"] = red
        out["cg"] = cg
    return out


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
    # kernel times: FP64 apply, 16-bit applies, diagonal
    xr = torch.tensor(synth.rand_x(op.ndof, 1), device="cuda")
    y = torch.empty_like(xr)
    k64 = time_kernel(op, hexpa, xr, y, 30)
    out["apply_fp64"] = roof_row(op.ndof, op.nelem, p, q, 2, k64)
    s = torch.cuda.current_stream()
    xr32 = xr.float()
    y32 = torch.empty_like(xr32)
    ab16 = op.nelem * 6 * q ** 3 * 4 + op.nelem * (p + 1) ** 3 * 4 + 8 * op.ndof
    for name, fmt in (("fp16", hexpa.PA_LP_FP16), ("bf16", hexpa.PA_LP_BF16)):
        for _ in range(5):
            hexpa.pa_apply_lp(op.h, xr32, y32, fmt)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(30):
            hexpa.pa_apply_lp(op.h, xr32, y32, fmt)
        e1.record(s)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / 30
        out[f"apply_{name}"] = {"ms_with_fill": ms, "alg_bytes": ab16,
                                "hbm_frac": ab16 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}
    d = torch.empty_like(xr)
    hexpa.pa_diag(op.h, d)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(10):
        hexpa.pa_diag(op.h, d)
    e1.record(s)
    torch.cuda.synchronize()
    out["diag_ms"] = e0.elapsed_time(e1) / 10
    out["diag_in_applies"] = out["diag_ms"] / k64
    log(f"C4 applies: fp64 {k64:.4f} ms, fp16 {out['apply_fp16']['ms_with_fill']:.4f} ms, "
        f"bf16 {out['apply_bf16']['ms_with_fill']:.4f} ms; diag {out['diag_ms']:.4f} ms")
    # normwise error of the 16-bit apply against the FP64 apply (unconstrained operator) for
    # a rough input (x ~ U[-1,1]) and a smooth one (the manufactured x*): rounding the
    # interpolated tile before differentiating costs more, relative to |A x|, when A x is small
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
    FCG on b = A_c x*_d), then on held-out draws 200.. compare FP64 Jacobi-PCG, FCG with
    coarse correction + Jacobi ("without the network") and FCG with coarse correction +
    network, each to 1e-8 from x = 0."""
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
    # what each part contributes: the coarse level (without the network) and the network on top
    out["speedup_coarse_jacobi_vs_jacobi"] = out["jacobi"]["seconds_mean"] / out["coarse_jacobi"]["seconds_mean"]
    out["speedup_net_vs_coarse_jacobi"] = out["coarse_jacobi"]["seconds_mean"] / out["coarse_net"]["seconds_mean"]
    out["iter_ratio_net_vs_coarse_jacobi"] = out["coarse_jacobi"]["iters_mean"] / out["coarse_net"]["iters_mean"]
    lp.close()
    return out


def run_paper_operator(hexpa, n=48, steps=50):
    """The paper's own operator (the off-diagonal blocks of the acoustic operator, eq. (4)):
    pressure H1 p=4, velocity L2 p=3 (three components), Q1D=5, on the 48^3 perturbed mesh
    (7,189,057 pressure + 21,233,664 velocity DOFs): the fused kernel applying D and D^T in
    one pass, timed by HIP events, and one lumped-mass RK4 step (four applies)."""
    import torch
    import synth
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    m = hexpa.MixedOperator(mesh)
    g = torch.Generator(device="cuda")
    g.manual_seed(0)
    u = torch.rand(m.ndof_u, dtype=torch.float64, device="cuda", generator=g) * 2 - 1
    p = torch.rand(m.ndof_p, dtype=torch.float64, device="cuda", generator=g) * 2 - 1
    yu, yp = torch.empty_like(u), torch.empty_like(p)
    warm(lambda: m.apply(u, p, yu, yp), 0.3, 3)
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        m.apply(u, p, yu, yp)
    e1.record(s)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    nd = m.ndof_u + m.ndof_p
    # D (9 FP64 per point), the pressure map, read u and p, write yu and yp
    alg = m.nelem * 9 * 125 * 8 + m.nelem * 125 * 4 + 16 * (m.ndof_u + m.ndof_p)
    out = {"workload": f"{n}^3 perturbed hex mesh, pressure H1 p=4 (GLL), velocity L2 p=3 (Gauss-Legendre nodes, "
                       f"3 components), Q1D=5, rho=K=1", "ndof_pressure": m.ndof_p, "ndof_velocity": m.ndof_u,
           "elems_per_group": m.info["elems_per_block"], "apply_ms_with_fill": ms, "gdofs": nd / ms / 1e6,
           "alg_bytes": alg, "hbm_frac": alg / ms / 1e6 / HBM_PEAK_GBS,
           "paper_context": "GB200 DMMA Fused PA 46.60 GDOF/s, GH200 36.15 GDOF/s at 540 M DOFs (Table VI)"}
    m.rk4(u * 1e-3, p * 1e-3, 1e-4, 2)
    torch.cuda.synchronize()
    e0.record(s)
    m.rk4(u, p, 1e-5, 10)
    e1.record(s)
    torch.cuda.synchronize()
    out["rk4_step_ms"] = e0.elapsed_time(e1) / 10
    log(f"paper operator: fused apply {ms:.4f} ms = {out['gdofs']:.1f} GDOF/s ({100 * out['hbm_frac']:.1f} % of HBM roof), "
        f"RK4 step {out['rk4_step_ms']:.3f} ms")
    m.close()
    return out


def _oracle_assembled_apply(oracle, P, sub):
    """Element matrices of the listed elements (timed: assembly), then y = sum_e G_e^T A_e G_e x
    over them by the oracle's assembled apply, on a compact numbering of the DOFs they touch
    (timed: apply; median of three batches of repeats)."""
    import ctypes
    t0 = time.perf_counter()
    Ae = P.elem_matrices(sub)
    t_asm = time.perf_counter() - t0
    ed = P.elem_dofs[sub]
    uniq, local = np.unique(ed, return_inverse=True)
    local = np.ascontiguousarray(local.reshape(ed.shape), dtype=np.int32)
    xl = np.random.default_rng(7).uniform(-1, 1, uniq.size)
    yl = np.zeros(uniq.size)
    lib = oracle.lib()

    def once():
        lib.orc_apply_assembled(ctypes.c_int64(sub.size), ctypes.c_int(P.nd), Ae.ctypes.data_as(ctypes.c_void_p),
                                local.ctypes.data_as(ctypes.c_void_p), ctypes.c_int64(uniq.size),
                                xl.ctypes.data_as(ctypes.c_void_p), yl.ctypes.data_as(ctypes.c_void_p))

    t0 = time.perf_counter()
    once()
    t1 = max(time.perf_counter() - t0, 1e-6)
    reps = max(1, int(0.2 / t1))
    batches = []
    for _ in range(3):
        t0 = time.perf_counter()
        for _ in range(reps):
            once()
        batches.append((time.perf_counter() - t0) / reps)
    return t_asm, float(np.median(batches))


def cpu_baseline(orders, budget_s):
    """The oracle on the host: per order of the sweep, dense element matrices assembled by
    quadrature loops (OpenMP) for a random element sample, then the assembled apply
    (single-threaded as the oracle stands) on that sample; both extrapolated to the whole
    mesh by the element share."""
    import oracle
    import synth
    threads = oracle.num_threads()
    per = []
    for p, n in orders:
        mesh = synth.box_mesh(n, perturb=0.1, seed=0)
        P = oracle.Problem(mesh, p, p + 2, ops=oracle.DIFFUSION)
        rng = np.random.default_rng(11)
        trial = np.sort(rng.choice(P.nelem, threads, replace=False)).astype(np.int32)
        t0 = time.perf_counter()
        P.elem_matrices(trial)
        t_el = (time.perf_counter() - t0) / trial.size
        mem_cap = int(1e9 / (8 * P.nd * P.nd))  # at most 1 GB of element matrices
        k = int(min(P.nelem, mem_cap, max(threads, budget_s / len(orders) / max(t_el, 1e-9))))
        sub = np.sort(rng.choice(P.nelem, k, replace=False)).astype(np.int32)
        t_asm, t_app = _oracle_assembled_apply(oracle, P, sub)
        scale = P.nelem / k
        per.append({"p": p, "n": n, "ndof": P.ndof, "elements_sampled": k, "nelem": P.nelem,
                    "assembly_seconds_extrapolated": t_asm * scale, "apply_seconds_extrapolated": t_app * scale,
                    "apply_gdofs": P.ndof / (t_app * scale) / 1e9})
        log(f"oracle p={p}: {k} of {P.nelem} elements, assembly {t_asm:.2f} s, apply {t_app * 1e3:.2f} ms")
    total_dofs = sum(r["ndof"] for r in per)
    total_t = sum(r["apply_seconds_extrapolated"] for r in per)
    return {"value": total_dofs / total_t / 1e9, "unit": "GDOF/s", "cores": 1, "kind": "oracle",
            "sample": "per order of the diffusion sweep, a random element sample (seed 11) sized to the time budget "
                      "(at most 1 GB of element matrices): dense element matrices assembled by quadrature loops, "
                      "then applied as y = sum_e G_e^T A_e G_e x on that sample (single-threaded; median of three "
                      "batches); apply time extrapolated to the whole mesh by the element share; value = sum of "
                      "DOFs / sum of extrapolated apply times over the four orders",
            "assembly_threads": threads, "per_order": per}


def oracle_cg(n, p=4, q=6):
    """The oracle's Jacobi-PCG (assembled element matrices) to 1e-8 on the C2 problem at a
    reduced mesh size: manufactured right-hand side, Dirichlet box boundary."""
    import oracle
    import synth
    from oracle import solvers
    mesh = synth.box_mesh(n, perturb=0.1, seed=0)
    P = oracle.Problem(mesh, p, q, coeff=oracle.Coeff.sine(), ops=oracle.DIFFUSION)
    ess = oracle.box_boundary(n, p).astype(bool)
    t0 = time.perf_counter()
    A = oracle.Assembled(P)
    t_asm = time.perf_counter() - t0
    b = np.where(ess, 0.0, P.load(synth.f_manufactured(P.qpoints().reshape(-1, 3)).reshape(P.nelem, -1)))
    Ac = solvers.constrained(A.apply, ess)
    dinv = 1.0 / solvers.constrained_diag(P.diag(), ess)
    t0 = time.perf_counter()
    x, it, rel, true, _ = solvers.pcg(Ac, b, lambda r: dinv * r, rtol=1e-8)
    t = time.perf_counter() - t0
    return {"mesh": f"{n}^3", "ndof": P.ndof, "iters": it, "seconds": t, "rel_res_true": float(true),
            "assembly_seconds": t_asm, "assembly_threads": oracle.num_threads(), "apply_threads": 1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--warm-seconds", type=float, default=1.0,
                    help="untimed applies for at least this long before the timed steps (sustained clocks)")
    ap.add_argument("--orders", default="2,4,6,8", help="orders of the headline sweep (profiling runs)")
    ap.add_argument("--cpu-budget", type=float, default=20.0, help="seconds of oracle CPU work (0 = skip)")
    ap.add_argument("--cg-reduced-n", type=int, default=12, help="mesh of the oracle's PCG beside the GPU's")
    ap.add_argument("--no-mass", action="store_true")
    ap.add_argument("--no-c2", action="store_true", help="skip the 48^3 leg (kernel matrix, energy, CG)")
    ap.add_argument("--no-cg", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--no-paper-operator", action="store_true", help="skip the mixed H1 x L2 acoustic operator")
    ap.add_argument("--no-matrix", action="store_true", help="skip the unfused/fused/matrix-free kernel matrix")
    ap.add_argument("--no-energy", action="store_true", help="skip the MDOF/W measurement")
    ap.add_argument("--learned-train", type=int, default=200, help="training draws of the learned preconditioner")
    ap.add_argument("--learned-held", type=int, default=20, help="held-out draws of the learned comparison")
    ap.add_argument("--learned-weights", default=None, help="load parameters from this file instead of training")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 2 GiB device copy (for HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)

    import torch
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

    want = {int(v) for v in args.orders.split(",")}
    orders = tuple((p, n) for p, n in SWEEP if p in want)
    wall, total_dofs, rows = run_headline(hexpa, args.steps, args.warmup, args.warm_seconds, orders)
    ms_step = 1e3 * wall / args.steps
    value = total_dofs * args.steps / wall / 1e9
    log(f"timed {args.steps} steps: {ms_step:.4f} ms/step, {value:.2f} GDOF/s")
    dom = max(rows, key=lambda r: r["kernel_ms"])  # the kernel with the largest share of a step
    pd, qd = dom["p"], dom["q1d"]
    stream = stream_read_gbps()
    dom_gbs = dom["alg_bytes"] / (dom["kernel_ms"] * 1e-3) / 1e9
    log(f"plain device-wide read on this machine: {stream:.0f} GB/s")
    out = {
        "metric": METRIC, "value": value, "unit": "GDOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "fp64 PA diffusion apply order sweep: p=2,4,6,8 with Q=p+2 on 155^3/78^3/52^3/40^3 "
                               "perturbed hex meshes of the unit cube (about 30 M DOFs each), kappa=1, x~U[-1,1]; "
                               "one step = one apply at each order",
                   "orders": [r["p"] for r in rows], "ndof_per_step": total_dofs},
        "roofline": {"bound": "hbm", "achieved": dom_gbs,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": dom["hbm_frac"],
                     "traffic": measured_traffic(f"k_apply_c3_p{pd}_diffusion_{dom['variant']}_hbm_traffic"),
                     "kernel": f"k_apply<D={pd + 1},Q={qd},diffusion,{dom['variant']}> (p={pd}, {dom['n']}^3)",
                     "alg_bytes_per_launch": dom["alg_bytes"], "alg_bytes_per_dof": dom["alg_bytes_per_dof"],
                     "kernel_ms_mean": dom["kernel_ms"], "fp64_frac": dom["fp64_frac"],
                     "stream_read_GBps": stream, "frac_of_stream_read": dom_gbs / stream},
        "sweep": rows,
    }
    if not args.no_mass:
        out["sweep_mass"] = run_mass_sweep(hexpa, orders)
    if not args.no_paper_operator:
        out["paper_operator"] = run_paper_operator(hexpa)
    if not args.no_c2:
        out["c2"] = run_c2(hexpa, args)
    if not args.no_mixed:
        out["mixed"] = run_mixed(hexpa)
        log("mixed-precision comparison done")
    if not args.no_learned:
        out["learned"] = run_learned(hexpa, args.learned_train, args.learned_held, weights=args.learned_weights)
        log("learned-preconditioner comparison done")
    if args.cpu_budget > 0:
        log("CPU oracle baseline ...")
        out["cpu_baseline"] = cpu_baseline(orders, args.cpu_budget)
        if "c2" in out and "cg" in out["c2"]:
            out["c2"]["cg"]["oracle_reduced_mesh"] = oracle_cg(args.cg_reduced_n)
            log(f"oracle PCG: {out['c2']['cg']['oracle_reduced_mesh']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
