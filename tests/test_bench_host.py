"""Host logic of the benchmark: the algorithmic work per launch behind the
roofline figures, the bound it picks, the counter records it accepts, and the
one-GPU guard.  No GPU is used."""
import os
import subprocess
import sys
from types import SimpleNamespace

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

# the medium workload's sizes: 16^3 cells, p = 6, 96^3 nodes, 7,948 (atom,
# cell) pairs of 8 projectors
MEDIUM = SimpleNamespace(ncells=4096, degree=6, npairs=7948, nbeta=8, ndof=2 * 96 ** 3)


def test_hx_flops_per_cell_and_pair():
    """24 n^2 + 16 n per (cell, vector) and 32 n n_beta per (pair, vector),
    n = (p + 1)^3: one cell, one pair, one vector at p = 1 (n = 8)."""
    p = SimpleNamespace(ncells=1, degree=1, npairs=1, nbeta=4)
    assert bench.hx_flops(p, 1) == (24 * 64 + 16 * 8, 32 * 8 * 4)
    loc, nl = bench.hx_flops(MEDIUM, 576)
    assert loc == 4096 * 576 * (24 * 343 ** 2 + 16 * 343)
    assert nl == 7948 * 576 * 32 * 343 * 8


def test_filter_roofline_work_and_bound():
    """The filter's fused kernel: per step the H X flops (projection half
    excluded) and 40 B per dof and vector (32 B in the first step); at the
    medium size it is bound by HBM, and frac is the binding fraction."""
    iters, q, nsub = 20, 30, 576
    launches = iters * (q - 1) * 8
    t = launches * 2.18e-3
    r = bench.filter_roofline(MEDIUM, "bf16", nsub, q, iters, t, launches, "none")
    loc, nl = bench.hx_flops(MEDIUM, nsub)
    assert r["flops_per_launch"] == pytest.approx((loc + nl / 2) / 8)
    per_dof = (q - 2) * 40 + 32
    assert r["bytes_per_launch"] == pytest.approx(MEDIUM.ndof * nsub * per_dof / (q - 1) / 8)
    assert r["bound"] == "hbm" and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(r["bytes_per_launch"] / 2.18e-3 / 8e12)
    assert r["frac_mfma"] == pytest.approx(r["flops_per_launch"] / 2.18e-3 / 2.5e15)
    assert r["traffic"] is None  # no counter record for this workload name
    # in FP64 (64 B per dof and vector) the same kernel is bound by the MFMAs
    r64 = bench.filter_roofline(MEDIUM, "fp64", nsub, q, iters, t, launches, "none")
    assert r64["bound"] == "mfma" and r64["frac"] == pytest.approx(r64["frac_mfma"])


def test_cell_roofline_bound_switch():
    """Plain H X: 16 B (complex64) or 32 B (complex128) per dof and vector;
    bfloat16 at the medium size is MFMA-bound by this accounting."""
    loc, nl = bench.hx_flops(MEDIUM, 512)
    r = bench.cell_roofline(MEDIUM, "bf16", 512, 11.85, 8, "none")
    assert r["bound"] == "mfma"
    assert r["frac"] == pytest.approx((loc + nl / 2) / 8 / (11.85e-3 / 8) / 2.5e15)
    assert r["bytes_per_launch"] == pytest.approx(2 * MEDIUM.ndof * 512 * 8 / 8)


def test_measured_traffic_records(tmp_path, monkeypatch):
    """A counter record is used only for its own kernel variant, workload and
    vector count, and only while the kernel source still has the recorded
    hash (checked on a copy of the committed record and source)."""
    import shutil
    rec = "cell_kernel_bf16_epi_medium_counters.txt"
    src = os.path.join("paper_2605_30128_amd", "csrc", "cell_bf16.h")
    (tmp_path / "profiles").mkdir()
    shutil.copy(os.path.join(ROOT, "profiles", rec), tmp_path / "profiles" / rec)
    os.makedirs(tmp_path / os.path.dirname(src))
    shutil.copy(os.path.join(ROOT, src), tmp_path / src)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    got = bench.measured_traffic("bf16", "medium", 576, variant="epi")
    if got is not None:  # the committed record matches the committed kernel
        assert 7e9 < got < 9e9
    assert bench.measured_traffic("bf16", "medium", 512, variant="epi") is None
    assert bench.measured_traffic("bf16", "slab", 576, variant="epi") is None
    assert bench.measured_traffic("bf16", "medium", 576) is None
    # a record whose hash matches its source is used; an edited source voids it
    import hashlib
    import json
    lines = open(tmp_path / "profiles" / rec).read().splitlines()
    r = json.loads([x for x in lines if x.startswith("TRAFFIC ")][-1][len("TRAFFIC "):])
    r["source_sha256"] = hashlib.sha256(open(tmp_path / src, "rb").read()).hexdigest()
    with open(tmp_path / "profiles" / rec, "a") as f:
        f.write("TRAFFIC " + json.dumps(r) + "\n")
    kib = r["fetch_kib_per_launch"] * r["fetch_scale"] + r["write_kib_per_launch"] * r["write_scale"]
    assert bench.measured_traffic("bf16", "medium", 576, variant="epi") == pytest.approx(1024 * kib)
    with open(tmp_path / src, "a") as f:
        f.write("// edited\n")
    assert bench.measured_traffic("bf16", "medium", 576, variant="epi") is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
