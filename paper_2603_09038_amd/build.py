"""Build libhexpa.so for gfx950 with hipcc (in-tree, next to this file).

Each source is compiled to its own object in parallel; k_apply.hip is compiled once
per polynomial order (-DHEXPA_APPLY_P=p) so the 8 orders build concurrently.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libhexpa.so")
ARCH = "gfx950"

HIPFLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-munsafe-fp-atomics",
    # packed FP32 instructions are kept out of every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
]


def _units():
    units = []
    for p in range(1, 9):
        units.append(("k_apply.hip", f"k_apply_p{p}.o", [f"-DHEXPA_APPLY_P={p}"]))
    for src in ("k_setup.hip", "k_diag.hip", "k_vec.hip", "k_debug.hip", "k_nn.hip", "noalloc.hip", "k_mixed.hip"):
        units.append((src, src.replace(".hip", ".o"), []))
    for src in ("api.cpp", "tables.cpp", "learned.cpp", "mixed.cpp"):
        units.append((src, src.replace(".cpp", ".o"), ["-x", "hip"]))
    return units


def _compile(unit, quiet):
    src, obj, extra = unit
    out = os.path.join(OBJ, obj)
    cmd = ["hipcc", "-c"] + HIPFLAGS + extra + [os.path.join(CSRC, src), "-o", out]
    if not quiet:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
    err = "\n".join(ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip())
    return out, err


def build(quiet=False, jobs=None):
    os.makedirs(OBJ, exist_ok=True)
    jobs = jobs or min(8, os.cpu_count() or 4)
    objs = []
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for out, err in ex.map(lambda u: _compile(u, quiet), _units()):
            objs.append(out)
            if err and not quiet:
                print(err, flush=True)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = ["hipcc", "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    if not quiet:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(quiet="-q" in sys.argv)
