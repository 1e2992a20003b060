"""Host-side contract of bench.py (no GPU): the one-GPU refusal and the algorithmic byte
model behind the roofline fraction."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_alg_bytes_counts_each_stream_once():
    # one p=2 element (27 DOFs), Q=4: D is [ncomp][Q^3] FP64, the map d^3 int32, x read and
    # y written once per DOF
    nelem, ndof, p, q = 1, 27, 2, 4
    for ops, ncomp in ((1, 1), (2, 6), (3, 7)):
        d_bytes = ncomp * 64 * 8
        assert bench.alg_bytes(ndof, nelem, p, q, ops) == d_bytes + 27 * 4 + 2 * 8 * 27
    # a 155^3 p=2 diffusion mesh: the headline's dominant kernel, 12.32 GB per launch
    n, p = 155, 2
    ab = bench.alg_bytes((n * p + 1) ** 3, n ** 3, p, p + 2, 2)
    assert abs(ab / 1e9 - 12.323) < 1e-3
