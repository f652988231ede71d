"""Benchmark of the R-ChFSI hot path on one MI355X.

A step is one R-ChFSI iteration (Algorithm RChFSI) on the medium workload:
Chebyshev filter of degree q in the mixed precision (the filter's H D^-1 Z
products), recovery, H Y and M Y in double, Cholesky-QR2, Rayleigh-Ritz and
the double-precision residual.  `value` is the number of H X dof-vectors
the timed steps processed per second (q products of the nsub-column block per
iteration), i.e. whole-job H X throughput including the Rayleigh-Ritz stage.
Isolated H X throughputs per precision, the double-precision iteration
time, the roofline of the dominant kernel (`roofline`: the filter's fused
cell kernel, timed with device events inside the timed iterations; the plain
H X kernel's is `roofline_hx`) and the CPU oracle baseline are reported
beside it, together with the block floating-point codec's
throughput and the Poisson workload (matrix-free K x throughput with its
roofline, PCG time to an absolute residual of 1e-10).

python bench.py [--gpus 1] [--steps K] [--warmup W] [--prec bf16|fp32]
python bench.py --poisson-only | --slab-only | --hx-only | --iter-only | --converge [--precs fp64,bf16,fp32]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"fp64": 78.6e12, "fp32": 157.3e12, "bf16": 2.5e15, "hbm": 8.0e12}
CSIZE = {"fp64": 16, "fp32": 8, "bf16": 8}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def hx_flops(p, nvec):
    """Algorithmic flops of one H X: local 24n^2 + 16n per cell and vector
    (K X, Phi X and Phi^T T on four real columns, 2x2 spin term), nonlocal
    32 n nbeta per (atom, cell) pair and vector (projection and apply)."""
    n = (p.degree + 1) ** 3
    local = p.ncells * nvec * (24 * n * n + 16 * n)
    nonloc = p.npairs * nvec * 32 * n * p.nbeta
    return local, nonloc


def _omp():
    """The OpenMP runtime the oracle library runs on (thread count control)."""
    import ctypes
    lib = ctypes.CDLL("libgomp.so.1")
    lib.omp_get_max_threads.restype = ctypes.c_int
    return lib


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(p, nvec=4, c0_iters=10):
    """The oracle timed on the host: H X on the medium mesh with all threads
    (the reported value) and with one thread, and the C0 (tiny) R-ChFSI
    solve for c0_iters iterations with all threads."""
    import numpy as np

    import oracle
    from paper_2605_30128_amd import synth
    oracle.build(force=False)
    omp = _omp()
    threads = omp.omp_get_max_threads()
    o = oracle.Oracle(p)
    X = synth.random_block(p.ndof, nvec, 9001)
    t0 = time.perf_counter()
    o.apply_H(X)
    dt = time.perf_counter() - t0
    omp.omp_set_num_threads(1)
    t0 = time.perf_counter()
    o.apply_H(X[:, :1].copy())
    dt1 = time.perf_counter() - t0
    omp.omp_set_num_threads(threads)
    del o, X
    cfg = synth.CONFIGS["tiny"]
    pt = synth.make_config("tiny")
    ot = oracle.Oracle(pt)
    lmax = ot.lanczos(20, synth.random_block(pt.ndof, 1, 2000)[:, 0])
    X0 = synth.random_block(pt.ndof, cfg["nsub"], 2001)
    t0 = time.perf_counter()
    r = ot.chfsi(X0, cfg["n_wanted"], cfg["cheb_degree"], lmax, tol=0.0, max_iter=c0_iters)
    dtc = time.perf_counter() - t0
    return {"value": p.ndof * nvec / dt / 1e9, "unit": "GDoF*vec/s", "cores": threads, "kind": "oracle",
            "sample": f"one H X of {nvec} vectors on the full medium mesh ({p.ndof} dofs), projector tables "
                      f"included, {dt:.1f} s with {threads} threads",
            "cpu_model": cpu_model(),
            "one_thread": {"value": p.ndof / dt1 / 1e9, "unit": "GDoF*vec/s", "cores": 1,
                           "sample": f"one H X of 1 vector on the medium mesh, {dt1:.1f} s"},
            "c0_solve": {"iterations": int(r["iters"]), "seconds": dtc, "sec_per_iter": dtc / max(r["iters"], 1),
                         "cores": threads,
                         "sample": f"tiny (C0) R-ChFSI, {cfg['nsub']} columns, degree {cfg['cheb_degree']}, "
                                   f"{r['iters']} iterations from the seeded start block"}}


def c0_gpu(iters=10):
    """The C0 (tiny) R-ChFSI solve on the GPU in FP64, iters fixed
    iterations from the same start block as the oracle's C0 timing."""
    import torch

    from paper_2605_30128_amd import binding, synth
    cfg = synth.CONFIGS["tiny"]
    p = synth.make_config("tiny")
    op = binding.Chfsi(p, max_nvec=cfg["nsub"])
    X = torch.from_numpy(synth.random_block(p.ndof, cfg["nsub"], 2001)).cuda()
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, 2000)[:, 0])
    out = op.solve(X, cfg["n_wanted"], cfg["cheb_degree"], prec="fp64", max_iter=iters, fixed_iters=True, v0=v0)
    return {"iterations": iters, "sec_per_iter_median": out["t_iter_median"], "seconds": out["t_total"],
            "prec": "fp64"}


MID = dict(ncell=(8, 8, 8), box=(12.0, 12.0, 12.0), degree=6, nwells=8, natoms=8, nbeta=8, seed=1010)


def gate_leg(precs=("fp64", "fp32", "bf16"), n_wanted=64, nsub=72, degree=30, tol=1e-8):
    """Mixed precision against FP64 to convergence at a mid-size shape (the
    medium mesh's cell size and degree on 8^3 cells, 110,592 nodes, 8 atoms
    x 8 projectors): each precision converges the same start block to the
    max wanted residual tol, and the wanted eigenvalues are compared with
    the FP64 run (the 1e-9 Ha gate)."""
    import numpy as np
    import torch

    from paper_2605_30128_amd import binding, synth
    p = synth.make_problem(**MID)
    op = binding.Chfsi(p, max_nvec=nsub)
    X0 = synth.random_block(p.ndof, nsub, 1011)
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, 1012)[:, 0])
    res, eig = {}, {}
    for prec in precs:
        X = torch.from_numpy(X0).cuda()
        r = op.solve(X, n_wanted, degree, prec=prec, tol=tol, max_iter=300, v0=v0, rr_mode=2)
        eig[prec] = r["eigvals"]
        res[prec] = {"iterations": r["iters"], "converged": r["converged"], "max_res": r["max_res"],
                     "sec_per_iter_median": r["t_iter_median"], "seconds": r["t_total"]}
        if prec != "fp64" and "fp64" in eig:
            res[prec]["max_abs_eig_diff_vs_fp64"] = float(np.abs(r["eigvals"] - eig["fp64"]).max())
        log(f"[bench] gate {prec}: {r['iters']} iterations to {r['max_res']:.2e}, "
            f"{r['t_iter_median'] * 1e3:.1f} ms/iter" +
            (f", max |dlambda| vs fp64 {res[prec]['max_abs_eig_diff_vs_fp64']:.2e} Ha"
             if "max_abs_eig_diff_vs_fp64" in res[prec] else ""))
    del op
    torch.cuda.empty_cache()
    return {"shape": f"8x8x8 cells of 1.5 bohr, p=6, {p.nnodes} nodes, {p.natoms} atoms x {p.nbeta} projectors, "
                     f"{n_wanted} wanted in {nsub} columns, Chebyshev degree {degree}, tol {tol:g}",
            "gate_ha": 1e-9, **res}


def cell_roofline(p, prec, nvec, ms_cell, launches, config):
    """Roofline of the cell-operator kernel: algorithmic flops (local plus the
    apply half of the spin-orbit term) and bytes (read X, write Y once) per
    launch over the device-event launch time."""
    loc, nl = hx_flops(p, nvec)
    flops_launch = (loc + nl / 2) / launches  # the projection half runs in the coefficient kernels
    bytes_launch = 2 * p.ndof * nvec * CSIZE[prec] / launches
    t_launch = ms_cell * 1e-3 / launches
    if flops_launch / PEAK[prec] >= bytes_launch / PEAK["hbm"]:
        roof = {"bound": "mfma", "achieved": flops_launch / t_launch / 1e12, "peak": PEAK[prec] / 1e12,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": bytes_launch / t_launch / 1e9, "peak": PEAK["hbm"] / 1e9,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(prec, config, nvec)
    roof["kernel"] = f"cell_kernel ({prec}), avg of {launches} colour launches per H X, {nvec} vectors"
    roof["flops_per_launch"] = flops_launch
    roof["bytes_per_launch"] = bytes_launch
    roof["ms_per_launch"] = t_launch * 1e3
    return roof


def filter_roofline(p, prec, nsub, degree, iters, t_cell, launches, config):
    """Roofline of the filter's cell-operator kernel (the fused recurrence
    variant, the dominant kernel of an R-ChFSI iteration) from device events
    around its launches inside the timed iterations.  Algorithmic work per
    filter step: the H D^-1 Z_k flops (local plus the apply half of the
    spin-orbit term) and the bytes of reading Z_k, Z_{k-1} (from the second
    step on) and R (complex128) and writing Z_{k+1} once: 40 B per dof and
    vector in FP32/BF16 (32 B in the first step), 64 B in FP64."""
    loc, nl = hx_flops(p, nsub)
    cz = CSIZE[prec]
    nsteps = iters * (degree - 1)
    flops = nsteps * (loc + nl / 2)
    per_dof = (degree - 2) * (3 * cz + 16) + (2 * cz + 16)  # per dof and vector, one filter
    bytes_ = iters * p.ndof * nsub * per_dof
    t_launch = t_cell / launches
    flops_launch, bytes_launch = flops / launches, bytes_ / launches
    if flops_launch / PEAK[prec] >= bytes_launch / PEAK["hbm"]:
        roof = {"bound": "mfma", "achieved": flops_launch / t_launch / 1e12, "peak": PEAK[prec] / 1e12,
                "unit": "TFLOP/s"}
    else:
        roof = {"bound": "hbm", "achieved": bytes_launch / t_launch / 1e9, "peak": PEAK["hbm"] / 1e9,
                "unit": "GB/s"}
    roof["frac"] = roof["achieved"] / roof["peak"]
    roof["traffic"] = measured_traffic(prec, config, nsub, variant="epi")
    roof["kernel"] = (f"cell_kernel ({prec}, fused recurrence), the filter's product in the timed iterations: "
                      f"{launches} launches ({nsteps} steps x colours), {nsub} columns")
    roof["flops_per_launch"] = flops_launch
    roof["bytes_per_launch"] = bytes_launch
    roof["ms_per_launch"] = t_launch * 1e3
    roof["frac_mfma"] = flops_launch / t_launch / PEAK[prec]
    roof["frac_hbm"] = bytes_launch / t_launch / PEAK["hbm"]
    return roof


def slab_leg(nvec=256, degree=40, reps=3, precs=("fp64", "fp32", "bf16"), filters=True):
    """The largest one-GPU share (periodic slab, 32 x 32 x 24 cells, p = 7,
    8,429,568 nodes, 256 atoms x 8 projectors), one block of nvec vectors:
    H X in FP64, FP32 and bfloat16 with the cell kernel's roofline, and the
    degree-40 filter pass over one block of wavefunctions in bfloat16
    (nvec columns), FP32 and FP64 (nvec/2 columns; half is the widest FP64
    block beside the other buffers in 288 GB) on synthetic X, R and Ritz
    values."""
    import numpy as np
    import torch

    from paper_2605_30128_amd import binding, synth
    t0 = time.perf_counter()
    p = synth.make_config("slab")
    log(f"[bench] slab generated: {p.ndof} dofs, {p.npairs} pairs in {time.perf_counter() - t0:.0f}s")
    op = binding.Chfsi(p, max_nvec=nvec, filter_block=nvec, filter_prec="bf16")
    out = {"nodes": p.nnodes, "dofs": p.ndof, "cells": p.ncells, "degree": p.degree, "vectors": nvec,
           "hx_gdofvec_per_s": {}, "hx_profile_ms": {}, "roofline": {}}
    X = synth.device_block(p.ndof, nvec, 801, dtype=torch.complex128 if "fp64" in precs else torch.complex64)
    for prec in precs:
        if prec != "fp64" and X.dtype == torch.complex128:
            X = X.to(torch.complex64)
            torch.cuda.empty_cache()
        Y = torch.empty_like(X)
        op.apply_H(X, prec=prec, Y=Y)
        r = [op.profile_apply_H(X, prec=prec, Y=Y) for _ in range(reps)]
        cell, coef, tot = (float(np.median([v[i] for v in r])) for i in range(3))
        out["hx_gdofvec_per_s"][prec] = p.ndof * nvec / (tot * 1e-3) / 1e9
        out["hx_profile_ms"][prec] = dict(ms_cell=cell, ms_coeff=coef, ms_total=tot, launches=r[0][3])
        out["roofline"][prec] = cell_roofline(p, prec, nvec, cell, r[0][3], "slab")
        log(f"[bench] slab H X {prec}: {tot:.1f} ms ({cell:.1f} cell) -> {out['hx_gdofvec_per_s'][prec]:.2f} "
            f"GDoF*vec/s, {out['roofline'][prec]['frac']:.3f} of the {out['roofline'][prec]['bound']} roof")
        del Y
    del X
    torch.cuda.empty_cache()
    if not filters:
        return out
    v0 = synth.device_block(p.ndof, 1, 802)[:, 0].contiguous()
    lmax = op.estimate_bounds(v0, 20)
    del v0
    Xf = synth.device_block(p.ndof, nvec, 803)
    R = synth.device_block(p.ndof, nvec, 804)
    R.mul_(1e-3)
    ritz = torch.linspace(-1.0, 2.0, nvec, dtype=torch.float64)
    bounds = [-1.0, 2.0, lmax]
    filt = {}
    for prec, ncol in (("bf16", nvec), ("fp32", nvec // 2), ("fp64", nvec // 2)):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        op.filter(Xf, ritz, R, degree, bounds, prec=prec, Y=Xf, nvec=ncol)
        ev[1].record()
        torch.cuda.synchronize()
        sec = ev[0].elapsed_time(ev[1]) * 1e-3
        filt[prec] = {"columns": ncol, "seconds": sec, "sec_per_column": sec / ncol,
                      "hx_gdofvec_per_s": (degree - 1) * p.ndof * ncol / sec / 1e9}
        log(f"[bench] slab filter {prec}: degree {degree}, {ncol} columns in {sec:.2f} s "
            f"({filt[prec]['hx_gdofvec_per_s']:.2f} GDoF*vec/s of H X)")
    filt["bf16_speedup_per_column"] = filt["fp64"]["sec_per_column"] / filt["bf16"]["sec_per_column"]
    filt["fp32_speedup_per_column"] = filt["fp64"]["sec_per_column"] / filt["fp32"]["sec_per_column"]
    filt["lambda_max"] = lmax
    out["filter_degree40"] = filt
    del Xf, R, op
    torch.cuda.empty_cache()
    return out


def adjoint_leg(op, p, nvec, reps=3):
    """The field adjoint of H X (dV, dB at the quadrature points for a pair
    X, G of nvec columns) in FP64 and FP32 with device events: its work per
    cell and vector is the two interpolations Phi X and Phi G on four real
    columns (16 n^2 flops) and the four spin sums per quadrature point (32 n);
    its bytes are reading X and G once."""
    import numpy as np
    import torch

    from paper_2605_30128_amd import synth
    n = (p.degree + 1) ** 3
    flops = p.ncells * nvec * (16 * n * n + 32 * n)
    out = {}
    for prec, dt in (("fp64", torch.complex128), ("fp32", torch.complex64)):
        X = synth.device_block(p.ndof, nvec, 7301, dtype=dt)
        G = synth.device_block(p.ndof, nvec, 7302, dtype=dt)
        op.adjoint(X, G, prec=prec, want_dX=False)
        ts = []
        for _ in range(reps):
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
            ev[0].record()
            op.adjoint(X, G, prec=prec, want_dX=False)
            ev[1].record()
            torch.cuda.synchronize()
            ts.append(ev[0].elapsed_time(ev[1]) * 1e-3)
        t = float(np.median(ts))
        out[prec] = {"ms": t * 1e3, "tflops": flops / t / 1e12, "frac_mfma": flops / t / PEAK[prec],
                     "bytes_hbm_frac": 2 * p.ndof * nvec * CSIZE[prec] / t / PEAK["hbm"]}
        log(f"[bench] adjoint fields {prec}: {t * 1e3:.1f} ms, {flops / t / 1e12:.2f} TFLOP/s, "
            f"{out[prec]['frac_mfma']:.3f} of the MFMA peak")
        del X, G
    torch.cuda.empty_cache()
    return out


def bfp_throughput(n=1 << 28, reps=5):
    """Device-event throughput of the block floating-point codec on n float
    values (1 GiB), per rate: bytes moved (floats and stream, read + write)
    per second and the fraction of the 8 TB/s HBM peak."""
    import torch

    from paper_2605_30128_amd import binding
    g = torch.Generator(device="cuda").manual_seed(11)
    x = torch.randn(n, generator=g, device="cuda", dtype=torch.float32)
    y = torch.empty_like(x)
    out = {}
    for nbits in (16, 12, 10):
        s = binding.bfp_encode(x, nbits)
        binding.bfp_decode(s, n, nbits, out=y)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        ev[0].record()
        for _ in range(reps):
            binding.bfp_encode(x, nbits, out=s)
        ev[1].record()
        for _ in range(reps):
            binding.bfp_decode(s, n, nbits, out=y)
        ev[2].record()
        torch.cuda.synchronize()
        moved = 4 * n + s.numel()
        te, td = ev[0].elapsed_time(ev[1]) / reps * 1e-3, ev[1].elapsed_time(ev[2]) / reps * 1e-3
        out[f"bfp{nbits}"] = {"encode_GBps": moved / te / 1e9, "decode_GBps": moved / td / 1e9,
                              "encode_frac_hbm": moved / te / PEAK["hbm"], "decode_frac_hbm": moved / td / PEAK["hbm"]}
        del s
    del x, y
    torch.cuda.empty_cache()
    return out


def kx_flops(degree, nq1, ncells):
    """Algorithmic flops of one sum-factorised K x (Sec. III-B1): per cell
    three interpolations to the Gauss points (n^3 q + n^2 q^2 + n q^3 FMAs),
    the three gradients and their transposes (6 q^4) and the three
    transposed interpolations (as many as the first three), 2 flops per FMA."""
    n, q = degree + 1, nq1
    return ncells * 2 * (2 * (n ** 3 * q + n ** 2 * q ** 2 + n * q ** 3) + 6 * q ** 4)


def poisson_leg(reps=50, pcg_solve=True):
    """The Poisson workload of the paper's electrostatics (Sec. III-B1): the
    matrix-free K x throughput (DoF/s) and its roofline on the medium mesh
    (p = 6) and on the largest one-GPU shape at p = 7 (the degree of the
    paper's K x comparison), and the PCG solve with a degree-5
    Chebyshev-Jacobi preconditioner to the absolute residual 1e-10 for a
    neutral Gaussian charge (f = 4 pi D rho, D the GLL-lumped mass)."""
    import math

    import numpy as np
    import torch

    from paper_2605_30128_amd import binding, synth
    out = {}
    for name in ("medium", "slab"):
        c = synth.CONFIGS[name]
        prob = synth.make_problem(ncell=c["ncell"], box=c["box"], degree=c["degree"], nwells=1, natoms=0,
                                  bfield="zero", soc=False, seed=c["seed"])
        ctx = binding.Chfsi(prob, max_nvec=1)
        M = ctx.nnodes
        g = torch.Generator(device="cuda").manual_seed(5)
        x = torch.randn(M, generator=g, device="cuda", dtype=torch.float64)
        y = torch.empty_like(x)
        for _ in range(3):
            ctx.apply_K(x, y)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(reps):
            ctx.apply_K(x, y)
        ev[1].record()
        torch.cuda.synchronize()
        t = ev[0].elapsed_time(ev[1]) / reps * 1e-3
        fl = kx_flops(prob.degree, prob.nq1, prob.ncells)
        rec = {"nodes": M, "cells": prob.ncells, "degree": prob.degree, "us_per_apply": t * 1e6,
               "gdof_per_s": M / t / 1e9,
               "roofline": {"bound": "alu", "achieved": fl / t / 1e12, "peak": PEAK["fp64"] / 1e12,
                            "unit": "TFLOP/s", "frac": fl / t / PEAK["fp64"], "traffic": kx_traffic(name),
                            "kernel": "apply_K: zero fill of y + kx_kernel (one launch)",
                            "flops_per_launch": fl, "hbm_GBps_16B_per_node": 16 * M / t / 1e9,
                            # the kernel applies every 1D operator in even/odd form, which
                            # halves the multiply-adds it executes
                            "executed_flops_per_launch": fl // 2, "frac_executed": fl / 2 / t / PEAK["fp64"]}}
        X = synth.node_coords(prob.ncell, prob.h, prob.degree)
        rho = synth.neutral_charge(X, prob.box, ncentres=8, seed=c["seed"])
        del X
        D = ctx.mass_diag()
        f = 4 * math.pi * D * torch.from_numpy(rho).cuda()
        del rho
        pcg = {}
        for deg in ((1, 5) if pcg_solve else ()):
            xs, rep, rc = ctx.poisson_solve(f, tol=1e-10, max_iter=20000, cheb_degree=deg, lanczos_steps=20)
            r = ctx.apply_K(xs) - (f - f.mean())
            pcg[f"cheb{deg}"] = {"status": rc, "iters": rep["iters"], "t_solve_s": rep["t_total"],
                                 "t_lanczos_s": rep["t_lanczos"],
                                 "ms_per_iter": 1e3 * (rep["t_total"] - rep["t_lanczos"]) / max(rep["iters"], 1),
                                 "res_norm": rep["res_norm"], "true_res_norm": float(r.norm()),
                                 "lambda_max": rep["lambda_max"]}
        rec["pcg_tol_abs_1e-10"] = pcg
        out[name] = rec
        log(f"[bench] poisson {name}: K x {t * 1e6:.1f} us ({M / t / 1e9:.1f} GDoF/s, "
            f"{fl / t / 1e12:.1f} TFLOP/s); PCG " +
            ", ".join(f"{k}: {v['iters']} it {v['t_solve_s'] * 1e3:.1f} ms" for k, v in pcg.items()))
        del ctx, x, y, f
        torch.cuda.empty_cache()
    return out


def cpu_poisson_baseline(name="medium"):
    """The oracle's K x (quadrature definition, numpy) on the medium mesh."""
    import numpy as np

    import oracle
    from oracle import poisson
    from paper_2605_30128_amd import synth
    oracle.build(force=False)
    c = synth.CONFIGS[name]
    prob = synth.make_problem(ncell=c["ncell"], box=c["box"], degree=c["degree"], nwells=1, natoms=0,
                              bfield="zero", soc=False, seed=c["seed"])
    K = poisson.Stiffness(oracle.Oracle(prob))
    x = np.random.default_rng(1).standard_normal(K.M)
    K.apply(x)
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        K.apply(x)
    dt = (time.perf_counter() - t0) / reps
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": K.M / dt / 1e9, "unit": "GDoF/s", "cores": threads, "kind": "oracle",
            "sample": f"{reps} K x on the {name} mesh ({K.M} nodes), {dt:.3f} s each"}


def kx_traffic(config):
    """HBM bytes per K x launch from the committed counter summary (calibrated
    FETCH_SIZE + WRITE_SIZE), or None if the kernel source changed since."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "kx_kernel_medium_slab_counters.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        if line.startswith("TRAFFIC "):
            rec = json.loads(line[len("TRAFFIC "):])
            if rec.get("config") != config:
                continue
            with open(os.path.join(ROOT, rec["source"]), "rb") as f:
                if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
                    return None
            return 1024.0 * (rec["fetch_kib_per_launch"] * rec["fetch_scale"] +
                             rec["write_kib_per_launch"] * rec["write_scale"])
    return None


def measured_traffic(prec, config, nvec, variant=""):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE runs, calibrated), or None when the
    summary is for another workload or the kernel source has changed since
    the counters were taken."""
    import hashlib
    tag = f"{prec}_{variant}" if variant else prec
    path = os.path.join(ROOT, "profiles", f"cell_kernel_{tag}_{config}_counters.txt")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("TRAFFIC "):
                rec = json.loads(line[len("TRAFFIC "):])
    if rec is None or rec.get("prec") != prec or rec.get("config") != config or rec.get("vectors") != nvec:
        return None
    with open(os.path.join(ROOT, rec["source"]), "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec["source_sha256"]:
            return None
    return 1024.0 * (rec["fetch_kib_per_launch"] * rec["fetch_scale"] + rec["write_kib_per_launch"] * rec["write_scale"])


def hellmann_feynman(op, p, cfg, prec="bf16", tol=1e-8, max_iter=400, h=1e-4, seed=7101):
    """Hellmann-Feynman check on the medium problem: L = sum of the n_wanted
    lowest Ritz values.  The adjoint with G = X (FP64 and FP32) gives dL/dV,
    dL/dB at the quadrature points; central differences of L re-solved at
    (V, B) +- h (dV, dB), each solve warm-started from the converged block,
    give the same directional derivative."""
    import numpy as np
    import torch

    from paper_2605_30128_amd import autograd, synth
    nw, nsub, q = cfg["n_wanted"], cfg["nsub"], cfg["cheb_degree"]
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, seed)[:, 0])
    X = torch.from_numpy(synth.random_block(p.ndof, nsub, seed + 1)).cuda()
    t0 = time.perf_counter()
    out = op.solve(X, nw, q, prec=prec, tol=tol, max_iter=max_iter, v0=v0, rr_mode=2)
    t_base = time.perf_counter() - t0
    log(f"[bench] hf: base solve {out['iters']} iterations to {out['max_res']:.2e} in {t_base:.1f} s")
    Xw = X[:, :nw].contiguous()
    grads = {pr: autograd.eigsum_grad(op, Xw if pr == "fp64" else Xw.to(torch.complex64), prec=pr)
             for pr in ("fp64", "fp32")}
    del Xw
    dV = torch.from_numpy(0.01 * synth.random_real(p.V.shape, seed + 2)).cuda()
    dB = torch.from_numpy(0.01 * synth.random_real(p.B.shape, seed + 3)).cuda()
    V0, B0 = torch.from_numpy(p.V).cuda(), torch.from_numpy(p.B).cuda()
    sums, its = [], []
    for sgn in (+1, -1):
        op.set_fields(V0 + sgn * h * dV, B0 + sgn * h * dB)
        Xs = X.clone()
        o2 = op.solve(Xs, nw, q, prec=prec, tol=tol, max_iter=max_iter, v0=v0, rr_mode=2)
        del Xs
        log(f"[bench] hf: solve at {sgn:+d}h, {o2['iters']} iterations to {o2['max_res']:.2e}")
        sums.append(float(np.sum(o2["eigvals"][:nw])))
        its.append(o2["iters"])
    op.set_fields(V0, B0)
    fd = (sums[0] - sums[1]) / (2 * h)
    res = {"shape": f"medium, {nw} wanted in {nsub} columns, Chebyshev degree {q}, {prec} filter, tol {tol}",
           "base_iterations": out["iters"], "base_seconds": t_base,
           "base_max_res": out["max_res"], "pm_iterations": its, "h": h, "fd": fd}
    for pr, (dVg, dBg) in grads.items():
        an = float((torch.sum(dVg.double() * dV) + torch.sum(dBg.double() * dB)).item())
        res[f"adjoint_{pr}"] = an
        res[f"rel_err_{pr}"] = abs(fd - an) / abs(an)
    del X
    torch.cuda.empty_cache()
    return res


def converge(op, p, cfg, precs, tol, max_iter, seed=7002, eig_file=None, rr_mode=1):
    """Runs Algorithm RChFSI to the tolerance in each precision from the same
    start block, one iteration per library call so that progress is printed,
    and compares the wanted eigenvalues with the FP64 run."""
    import numpy as np
    import torch

    from paper_2605_30128_amd import synth
    nsub, q, nw = cfg["nsub"], cfg["cheb_degree"], cfg["n_wanted"]
    X0 = synth.random_block(p.ndof, nsub, seed)
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, seed + 1)[:, 0])
    res = {}
    for prec in precs:
        rrm = rr_mode if prec != "fp64" else 1  # the FP64 reference keeps the FP64 rotation
        X = torch.from_numpy(X0).to("cuda", torch.complex128)
        t0 = time.perf_counter()
        out = op.solve(X, nw, q, prec=prec, tol=tol, max_iter=1, v0=v0, rr_mode=rrm)
        lmax, work, hist = out["bounds"][2], out["work"], [float(out["hist_res"][0])]
        it = 1
        while not out["converged"] and it < max_iter:
            out = op.solve(X, nw, q, prec=prec, tol=tol, max_iter=1, resume=True, work=work, lambda_max=lmax,
                           rr_mode=rrm)
            hist.append(float(out["max_res"]))
            it += 1
            log(f"[converge] {prec} iteration {it}: max residual {out['max_res']:.3e} "
                f"({time.perf_counter() - t0:.0f}s)")
        torch.cuda.synchronize()
        res[prec] = dict(iters=it, converged=bool(out["converged"]), seconds=time.perf_counter() - t0,
                         eig=out["eigvals"].copy(), hist=hist)
        if eig_file:
            # every wanted eigenvalue, so runs made in separate processes can be compared
            with open(eig_file.replace("{prec}", prec), "w") as f:
                json.dump({"prec": prec, "tol": tol, "iterations": it, "converged": bool(out["converged"]),
                           "seconds": res[prec]["seconds"], "residual_history": hist,
                           "eigvals": [float(v) for v in out["eigvals"]]}, f)
        log(f"[converge] {prec}: {it} iterations, converged={out['converged']}, {res[prec]['seconds']:.1f}s")
        del X
        torch.cuda.empty_cache()
    summary = {"tol": tol, "n_wanted": nw, "nsub": nsub, "degree": q}
    for prec in precs:
        r = res[prec]
        d = {"iterations": r["iters"], "converged": r["converged"], "seconds": r["seconds"],
             "residual_history": r["hist"]}
        if prec != "fp64" and "fp64" in res:
            d["max_abs_eig_diff_vs_fp64"] = float(np.abs(r["eig"] - res["fp64"]["eig"]).max())
        summary[prec] = d
    summary["eig_fp64_first8"] = res["fp64"]["eig"][:8].tolist() if "fp64" in res else None
    return summary


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="medium")
    ap.add_argument("--prec", default="bf16", choices=["bf16", "fp32", "fp64"])
    ap.add_argument("--hx-reps", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64-iter", action="store_true")
    ap.add_argument("--converge", action="store_true",
                    help="instead of timing: solve to --tol in fp64, bf16 and fp32 and compare eigenvalues")
    ap.add_argument("--hf", action="store_true",
                    help="only the Hellmann-Feynman check: re-solved eigenvalue sums vs the adjoint")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--max-iter", type=int, default=60)
    ap.add_argument("--precs", default="fp64,bf16,fp32", help="precisions of --converge")
    ap.add_argument("--rr-mode", type=int, default=2, choices=[0, 1, 2],
                    help="Rayleigh-Ritz of the mixed iterations: 1 FP64, 2 mixed-precision subspace rotation")
    ap.add_argument("--eig-file", default=None,
                    help="--converge: write each run's eigenvalues to this path ({prec} is replaced)")
    ap.add_argument("--hx-only", action="store_true",
                    help="only the H X products (for counter runs), after a 1 GiB fill and a 1 GiB sum that "
                         "calibrate the memory counters")
    ap.add_argument("--hx-precs", default="fp64,fp32,bf16")
    ap.add_argument("--no-poisson", action="store_true", help="skip the Poisson (K x, PCG) leg")
    ap.add_argument("--no-gate", action="store_true", help="skip the mid-size mixed-vs-FP64 convergence leg")
    ap.add_argument("--no-slab", action="store_true", help="skip the largest-share (slab) leg")
    ap.add_argument("--slab-only", action="store_true", help="run only the slab leg")
    ap.add_argument("--slab-precs", default="fp64,fp32,bf16", help="--slab-only: H X precisions")
    ap.add_argument("--slab-no-filter", action="store_true", help="--slab-only: H X only (for counter runs)")
    ap.add_argument("--poisson-only", action="store_true", help="run only the Poisson leg")
    ap.add_argument("--no-pcg", action="store_true", help="Poisson leg: K x only")
    ap.add_argument("--kx-reps", type=int, default=50)
    ap.add_argument("--adjoint-only", action="store_true",
                    help="only the field adjoint of H X in FP64 and FP32 (512 vectors)")
    ap.add_argument("--iter-only", action="store_true",
                    help="only the warm-up and timed R-ChFSI iterations (after the 1 GiB fill and sum that "
                         "calibrate the memory counters)")
    ap.add_argument("--calibrate", action="store_true",
                    help="with --poisson-only: run the 1 GiB fill and sum used to scale memory counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): this build has no multi-GPU path; "
              "the filter would shard over column blocks of X, see the design notes.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2605_30128_amd import binding, synth

    binding.load()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.poisson_only:
        if args.calibrate:
            # memory-counter calibration: a fill writes 2^30 bytes, a sum reads them
            a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
            a.fill_(1.0)
            a.sum().item()
            torch.cuda.synchronize()
            del a
        poi = poisson_leg(reps=args.kx_reps, pcg_solve=not args.no_pcg)
        if not args.no_cpu_baseline:
            poi["cpu_baseline"] = cpu_poisson_baseline()
        print(json.dumps({"poisson": poi}), flush=True)
        return
    if args.slab_only:
        if args.slab_no_filter:
            # memory-counter calibration: a fill writes 2^30 bytes, a sum reads them
            a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
            a.fill_(1.0)
            a.sum().item()
            torch.cuda.synchronize()
            del a
        print(json.dumps({"slab": slab_leg(precs=tuple(args.slab_precs.split(",")),
                                           filters=not args.slab_no_filter)}), flush=True)
        return
    cfg = synth.CONFIGS[args.config]
    t0 = time.perf_counter()
    p = synth.make_config(args.config)
    log(f"[bench] generated {args.config}: {p.ndof} dofs, {p.npairs} pairs in {time.perf_counter() - t0:.1f}s")
    nsub, nhx, q = cfg["nsub"], cfg["nvec_hx"], cfg["cheb_degree"]
    op = binding.Chfsi(p, max_nvec=max(nsub, nhx))
    log("[bench] setup done")
    if args.hf:
        print(json.dumps({"hellmann_feynman": hellmann_feynman(op, p, cfg, prec=args.prec, tol=args.tol)}),
              flush=True)
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": adjoint_leg(op, p, nhx)}), flush=True)
        return
    if args.converge:
        print(json.dumps({"convergence": converge(op, p, cfg, args.precs.split(","), args.tol, args.max_iter,
                                                  eig_file=args.eig_file, rr_mode=args.rr_mode)}), flush=True)
        return

    if args.hx_only or args.iter_only:
        # memory-counter calibration: a fill writes 2^30 bytes, a sum reads them
        a = torch.empty(2 ** 28, dtype=torch.float32, device="cuda")
        a.fill_(1.0)
        a.sum().item()
        torch.cuda.synchronize()
        del a

    # ---- isolated H X per precision (nhx vectors)
    hx = {}
    prof = {}
    for prec in [] if args.iter_only else args.hx_precs.split(","):
        dt = torch.complex128 if prec == "fp64" else torch.complex64
        X = torch.from_numpy(synth.random_block(p.ndof, nhx, 7001)).to("cuda", dt)
        Y = torch.empty_like(X)
        for _ in range(2):
            op.apply_H(X, prec=prec, Y=Y)
        torch.cuda.synchronize()
        reps = [op.profile_apply_H(X, prec=prec, Y=Y) for _ in range(args.hx_reps)]
        cell = float(np.median([r[0] for r in reps]))
        coef = float(np.median([r[1] for r in reps]))
        tot = float(np.median([r[2] for r in reps]))
        launches = reps[0][3]
        hx[prec] = p.ndof * nhx / (tot * 1e-3) / 1e9
        prof[prec] = dict(ms_cell=cell, ms_coeff=coef, ms_total=tot, launches=launches)
        log(f"[bench] H X {prec}: {tot:.2f} ms ({cell:.2f} cell, {coef:.2f} coeff) -> {hx[prec]:.2f} GDoF*vec/s")
        del X, Y
    torch.cuda.empty_cache()
    if args.hx_only:
        print(json.dumps({"hx_gdofvec_per_s": hx, "hx_profile_ms": prof}), flush=True)
        return

    # ---- the timed steps: R-ChFSI iterations
    n_wanted = cfg["n_wanted"]
    X = torch.from_numpy(synth.random_block(p.ndof, nsub, 7002)).to("cuda", torch.complex128)
    v0 = torch.from_numpy(synth.random_block(p.ndof, 1, 7003)[:, 0])
    out = op.solve(X, n_wanted, q, prec=args.prec, max_iter=max(args.warmup, 1), fixed_iters=True, v0=v0,
                   rr_mode=args.rr_mode)
    lmax = out["bounds"][2]
    work = out["work"]
    log(f"[bench] warmup done: residual {out['max_res']:.3e}, lambda_max {lmax:.3f}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = op.solve(X, n_wanted, q, prec=args.prec, max_iter=args.steps, fixed_iters=True, resume=True, work=work,
                   lambda_max=lmax, rr_mode=args.rr_mode, profile=True)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall / args.steps * 1e3
    value = args.steps * q * p.ndof * nsub / wall / 1e9
    log(f"[bench] {args.steps} {args.prec} iterations: {ms_step:.1f} ms/iter (filter {out['t_filter']:.3f}s, "
        f"rr {out['t_rr']:.3f}s), residual {out['max_res']:.3e}")
    roof = filter_roofline(p, args.prec, nsub, q, out["iters"], out["t_filter_cell"], out["filter_cell_launches"],
                           args.config)
    log(f"[bench] filter cell kernel: {roof['ms_per_launch']:.3f} ms per launch, {roof['frac']:.3f} of the "
        f"{roof['bound']} roof (mfma {roof['frac_mfma']:.3f}, hbm {roof['frac_hbm']:.3f})")
    if args.iter_only:
        print(json.dumps({"sec_per_iter": {args.prec: ms_step / 1e3}, "roofline": roof}), flush=True)
        return
    it64 = None
    if not args.no_fp64_iter and args.prec != "fp64":
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        o64 = op.solve(X, n_wanted, q, prec="fp64", max_iter=1, fixed_iters=True, resume=True, work=work,
                       lambda_max=lmax, rr_mode=1)
        torch.cuda.synchronize()
        it64 = time.perf_counter() - t1
        log(f"[bench] 1 fp64 iteration: {it64 * 1e3:.1f} ms (filter {o64['t_filter']:.3f}s)")
    it32 = None
    if not args.no_fp64_iter and args.prec != "fp32":
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        o32 = op.solve(X, n_wanted, q, prec="fp32", max_iter=1, fixed_iters=True, resume=True, work=work,
                       lambda_max=lmax, rr_mode=args.rr_mode)
        torch.cuda.synchronize()
        it32 = time.perf_counter() - t1
        log(f"[bench] 1 fp32 iteration: {it32 * 1e3:.1f} ms (filter {o32['t_filter']:.3f}s)")
    del X, work, out
    torch.cuda.empty_cache()

    # ---- roofline of the plain H X cell kernel (the timed iterations' fused kernel is `roof`)
    pr = args.prec
    roof_hx = cell_roofline(p, pr, nhx, prof[pr]["ms_cell"], prof[pr]["launches"], args.config)

    adj = adjoint_leg(op, p, nhx)
    bfp = bfp_throughput()
    log(f"[bench] bfp codec: " + ", ".join(f"{k} enc {v['encode_GBps']:.0f} / dec {v['decode_GBps']:.0f} GB/s"
                                           for k, v in bfp.items()))

    poi = None
    if not args.no_poisson:
        poi = poisson_leg()
        if not args.no_cpu_baseline:
            try:
                poi["cpu_baseline"] = cpu_poisson_baseline()
            except Exception as e:  # the baseline is a report, never the product
                log(f"[bench] cpu poisson baseline failed: {e}")

    del op
    torch.cuda.empty_cache()
    gate = None if args.no_gate else gate_leg()
    slab = None if args.no_slab else slab_leg()

    cpu = None
    if not args.no_cpu_baseline:
        try:
            cpu = cpu_baseline(p)
            cpu["c0_gpu"] = c0_gpu()
            log(f"[bench] cpu baseline: {cpu}")
        except Exception as e:  # the baseline is a report, never the product
            log(f"[bench] cpu baseline failed: {e}")

    res = {
        "metric": "GDoF*vec/s of H*X + sec/R-ChFSI iter, mixed vs FP64 at 1e-9 Ha eigen error",
        "value": value,
        "unit": "GDoF*vec/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": pr,
        "data": "synthetic",
        "config": {
            "workload": f"{args.config}: periodic cube {p.box[0]:g} bohr, {p.ncell[0]}x{p.ncell[1]}x{p.ncell[2]} "
                        f"cells, p={p.degree}, {p.ndof} complex spinor dofs, {p.natoms} atoms x {p.nbeta} SOC "
                        f"projectors, {nsub}-column subspace ({n_wanted} wanted), Chebyshev degree {q}",
            "filter_precision": pr,
            "rr_precision": "fp64" if args.rr_mode < 2 else "fp64 (subspace rotation fp64 diagonal / fp32 off-diagonal blocks)",
            "hx_vectors": nhx,
            "nsub": nsub,
        },
        "sec_per_iter": {pr: ms_step / 1e3, "fp64": it64, **({"fp32": it32} if it32 is not None else {})},
        "mixed_vs_fp64_gate": gate,
        "slab": slab,
        "hx_gdofvec_per_s": hx,
        "hx_profile_ms": prof,
        "roofline": roof,
        "roofline_hx": roof_hx,
        "adjoint": adj,
        "bfp_codec": bfp,
        "poisson": poi,
        "cpu_baseline": cpu,
    }
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
