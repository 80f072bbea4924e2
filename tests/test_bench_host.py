"""Host logic of the benchmark script: the algorithmic byte counts of the
roofline, the cells whose product reads a stored diagonal, the guard of the
profile-derived traffic, and the one-GPU contract."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1207_1571_amd import workloads as wl  # noqa: E402


def test_product_bytes_at_the_200_cube():
    """The 200^3 cavity: N = 8e6 cells, 3 * 200^2 * 199 internal faces, no
    explicit slice, the diagonal read only in the reference pin's slice.
    FP64: x and y (16 B), one 8-byte coefficient per face, 256 diagonals;
    FP32: x and y (8 B), one 4-byte coefficient per face, 256 row sums."""
    N, Fi = 200 ** 3, 3 * 200 * 200 * 199
    sell = {"explicit_entries": 0, "n_explicit_slices": 0}
    assert bench.algorithmic_bytes("pcg_spmv", N, Fi, sell, 256) == 128_000_000 + 2_048 + 191_040_000
    assert bench.algorithmic_bytes("pcg32_spmv", N, Fi, sell, 256) == 64_000_000 + 1_024 + 95_520_000
    # an explicit slice layout (random numbering) adds one int32 per entry,
    # two entries per internal face
    rnd = {"explicit_entries": 2 * Fi, "n_explicit_slices": N // 256}
    assert (bench.algorithmic_bytes("pcg_spmv", N, Fi, rnd, N)
            - bench.algorithmic_bytes("pcg_spmv", N, Fi, sell, N)) == 8 * Fi
    # the streaming kernels: 7 and 4 FP64 arrays per cell
    assert bench.algorithmic_bytes("pcg_update", N, Fi) == 56 * N
    assert bench.algorithmic_bytes("pcg_dir", N, Fi) == 32 * N


def test_diagonal_read_cells():
    """A cavity has no fixed-pressure patch: only the reference pin's slice
    reads its diagonals.  A duct fixes the pressure at its outlet x = L:
    every slice holding a cell of the last x-layer reads them; the slices
    are found here from the cell coordinates (index = x + nx (y + ny z))."""
    cav = wl.cavity((20, 20, 20), Re=10.0, dt=0.01)
    assert bench.diag_read_cells(cav, {"n_explicit_slices": 0}) == 256
    nx, ny, nz = 40, 12, 10
    duct = wl.duct((nx, ny, nz))
    y, z = np.meshgrid(np.arange(ny), np.arange(nz), indexing="ij")
    outlet = (nx - 1) + nx * (y + ny * z)
    slices = np.unique(outlet.ravel() // 256)
    assert bench.diag_read_cells(duct, {"n_explicit_slices": 0}) == min(nx * ny * nz, 256 * len(slices))


def test_traffic_records_are_keyed_to_the_kernel_source(monkeypatch):
    """Every traffic record under profiles/ parses and carries the fields the
    roofline uses; a record is only used while the kernel source is the one
    profiled."""
    import glob
    recs = []
    for f in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(f):
            if line.startswith("traffic-json:"):
                recs.append(json.loads(line.split(":", 1)[1]))
    assert recs
    for r in recs:
        assert {"kernel_class", "workload", "kernels_hip_sha256", "median_us", "bytes_per_working_launch"} <= set(r)
        assert r["median_us"] > 0 and r["bytes_per_working_launch"] > 0
    cls, wk = recs[0]["kernel_class"], recs[0]["workload"]
    monkeypatch.setattr(bench, "kernels_sha256", lambda: recs[0]["kernels_hip_sha256"])
    assert bench.measured_traffic(cls, wk) is not None
    monkeypatch.setattr(bench, "kernels_sha256", lambda: "0" * 64)
    assert bench.measured_traffic(cls, wk) is None
    assert bench.counter_GBps(None) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], cwd=ROOT,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
