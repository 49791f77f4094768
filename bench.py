#!/usr/bin/env python3
"""Throughput of FE cell kernels + CSR assembly on one MI355X.

Workload: P4 Lagrange mass + stiffness matrices on the unit cube split into
24^3 boxes x 6 Kuhn tetrahedra (82,944 cells, 35 dofs/cell), interior
vertices jittered +-0.25 h, 5% of cells flattened to aspect ratio 1e3,
collapsed Gauss-Jacobi quadrature of degree 8 (125 points), z = 1.  Both
matrices share one CSR pattern (912,673 rows, 67,338,433 nnz each).

One step = one FE_NUMERIC call of the library: cell kernels of both forms
(geometry, H formation, matrix-core contraction) and the deterministic CSR
assembly of both matrices, inputs resident in HBM.  The step runs a
geometry pass and one fused pass over the row-ownership schedule that
computes and writes both matrices; the two halves are also timed on their
own (FE_NUMERIC_GEOMETRY, FE_NUMERIC_FUSED) for the roofline of the fused
pass.  The mixed FP16/FP32
path is the reported value; the plain FP64 path is timed beside it on the
same mesh, and the relative Frobenius error of the mixed result against the
FP64 result is reported (the FP64 path itself matches the FP64 CPU oracle
to 1e-12 in the GPU tests).

The same line carries, under "action_vjp", the matrix-free action of
Algorithm 2 and its vector-Jacobian product on the P6 weighted-stiffness
workload (32^3 x 6 tetrahedra, 196,608 cells, 84 dofs/cell, 512-point rule,
kappa = exp(sin(2 pi x) cos(2 pi y) z) interpolated in P6, u and v ~ N(0,1)
in FP32): one step = y = A(kappa) u, then grad_u = A(kappa)^T v and
grad_kappa = v^T (dA/dkappa) u, in FP32 with the FP64 path beside it.

Under "mixed_degree": the batched mixed-degree workload (first 400,000
tetrahedra of the 41^3 x 6 mesh, degree p in 1..8 per cell with P(p) ~ 1/p,
quadrature degree 2p, mass form of a discontinuous space, cells in one
contiguous block per degree, one block-diagonal CSR of 1.14e9 entries): one
step = the numeric phase of all eight blocks (per-degree tiles from the
autotuner) replayed as one HIP graph, FP16 storage / FP32 accumulation, the
FP64 path beside it.

Under "hex_mass" and "hex_stiffness": the mass and Poisson forms on
hexahedra (the paper's boxed cells): 38^3 jittered trilinear hexahedra
(54,872 cells), Q4 (125 dofs/cell), the 125-point tensor Gauss-Legendre
rule, |det J| (mass) or G = |det J| J^-1 J^-T (Poisson) per quadrature
point; one step = FE_NUMERIC (mass: geometry pass + fused row-ownership
pass; Poisson: cell kernels + row gather into CSR), FP16 storage / FP32
accumulation, the FP64 path beside it.

Under "weighted_p6": the weighted P6 stiffness form div(kappa grad u) on the
32^3 x 6 mesh (196,608 cells, 84 dofs/cell, 512-point rule, kappa as above,
FP64 geometry) in BF16, FP16, FP32 and FP64 (the precision sweep): one step
= FE_NUMERIC (cell kernels with the coefficient at the points, then the row
gather into CSR); every mode's cell kernel is also timed alone for its
matrix-core roofline, and every mode's error is taken against the FP64
result.  The P4 line also carries the BF16 and split-FP16 modes under
"other_modes".

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peaks used for roofline fractions (MI355X published figures).
PEAK_HBM_GBS = 8000.0
PEAK_MFMA_TFLOPS = {"fp16": 2500.0, "bf16": 2500.0, "split": 2500.0, "fp32": 157.3, "fp64": 78.6}
# vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2 operations per lane (packed
# pair) x 2 flops per fused multiply-add x 2.4 GHz = 157.3 TFLOP/s, the
# published packed FP32 vector figure; packed half FMAs run at the same
# pair rate (unpacked FP32 is half of it, 78.6)
PEAK_VALU_TFLOPS = 157.3

# Measured HBM traffic (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a
# plain copy) of the dominant kernels, and the sources each was measured
# with (a figure is reported only for the code it was measured on).
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_pass_c2_fp16_traffic.txt")
KERNEL_SOURCES = ["fe_fused.h", "fe_cell_kernel.h", "fe_internal.h", "fe_cell_fp16.hip", "fe_csr.hip"]
CW_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cellwise_c3_fp16_traffic.txt")
CW_SOURCES = ["fe_cellwise.h", "fe_cell_kernel.h", "fe_internal.h", "fe_cell_fp16.hip"]
GATHER_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gather_c3_fp16_traffic.txt")
GATHER_SOURCES = ["fe_csr.hip", "fe_internal.h"]

WORKLOAD = ("P4 Lagrange mass+stiffness, 24^3 x 6 jittered Kuhn tetrahedra (82,944 cells, "
            "35 dofs/cell), 5% flattened to aspect 1e3, 125-point collapsed Gauss-Jacobi rule")


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    # the default window (100 timed steps after 50 untimed ones, about 0.1 s)
    # is long enough for the clocks to settle; 20 steps right after set-up
    # read about 10 % slow
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--precision", default="fp16", choices=["fp16", "bf16", "split", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--cpu-sample-cells", type=int, default=0,
                    help="cells of the oracle baseline sample (0 = the whole mesh)")
    ap.add_argument("--cpu-reps", type=int, default=3, help="oracle passes over the sample")
    ap.add_argument("--no-action", action="store_true",
                    help="skip the action / vector-Jacobian product measurement")
    ap.add_argument("--action-cpu-cells", type=int, default=0,
                    help="cells of the oracle baseline sample of the action step (0 = all)")
    ap.add_argument("--no-mixed", action="store_true",
                    help="skip the mixed-degree batch measurement")
    ap.add_argument("--mixed-cpu-cells", type=int, default=240000,
                    help="cells (first n of the mesh) of the oracle sample of the mixed batch")
    ap.add_argument("--no-hex", action="store_true",
                    help="skip the hexahedral mass measurement")
    ap.add_argument("--no-c3", action="store_true",
                    help="skip the weighted P6 stiffness precision sweep")
    ap.add_argument("--c3-cpu-cells", type=int, default=8192,
                    help="cells (first n) of the oracle sample of the weighted stiffness step")
    ap.add_argument("--hex-cpu-cells", type=int, default=10000,
                    help="cells (first n) of the oracle sample of the hexahedral mass step")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 256 MiB elementwise copy (x * 1.0), the reference "
                         "kernel for scaling hardware byte counters")
    return ap.parse_args()


def log(msg):
    """Progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


WARM_S = 0.25  # least wall time of untimed calls before a timed window


def time_steps(fn, steps, warmup):
    """Average ms per call of ``fn`` over ``steps`` calls, HIP events on the
    current stream (the stream the library launches on).  Untimed calls
    first: ``warmup`` of them, and more until WARM_S seconds have passed, so
    that the GPU clocks have left their idle state (a window timed right
    after host-side set-up reads up to 15 % slow)."""
    import torch
    t0 = time.perf_counter()
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    while time.perf_counter() - t0 < WARM_S:
        for _ in range(4):
            fn()
        torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(steps):
        fn()
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def cpu_baseline(mesh, sample_cells, reps):
    """The FP64 oracle (numeric phase: local matrices of both forms + CSR
    assembly) on the first ``sample_cells`` cells, ``reps`` passes, OpenMP
    over the host cores."""
    import oracle
    n = mesh.n_cells if sample_cells <= 0 else min(sample_cells, mesh.n_cells)
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
    tab = oracle.tabulation(3, mesh.degree, 8)
    cc, dm = mesh.cell_coords[:n], mesh.dofmap[:n]
    rp, ci = oracle.csr_pattern(dm, mesh.n_dofs)          # symbolic: not timed
    t0 = time.perf_counter()
    for _ in range(reps):
        for form in ("mass", "stiffness"):
            A = oracle.local_matrices(form, cc, mesh.degree, 8, nthreads=threads, tab=tab)
            oracle.assemble(dm, A, mesh.n_dofs, rp, ci)
            del A
    dt = (time.perf_counter() - t0) / reps
    # the same numeric phase on one thread, on the first 4,096 cells
    n1 = min(4096, n)
    rp1, ci1 = oracle.csr_pattern(dm[:n1], mesh.n_dofs)
    t0 = time.perf_counter()
    for form in ("mass", "stiffness"):
        A = oracle.local_matrices(form, cc[:n1], mesh.degree, 8, nthreads=1, tab=tab)
        oracle.assemble(dm[:n1], A, mesh.n_dofs, rp1, ci1)
        del A
    dt1 = time.perf_counter() - t0
    return {"value": n / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} of {mesh.n_cells} cells (first n), both forms, local matrices + CSR "
                      f"assembly (FP64, {threads} OpenMP threads), {reps} passes of {dt:.1f} s",
            "single_thread": {"value": n1 / dt1, "unit": "cells/s", "cores": 1,
                              "sample": f"first {n1} cells, one pass of {dt1:.1f} s"}}


def action_section(args, steps, warmup):
    """Action + VJP step on the P6 weighted-stiffness workload (FP32, FP64
    beside it), its matrix-core roofline and an oracle baseline sample."""
    import numpy as np
    import torch

    import oracle
    from fe_inputs import config_mesh, normal_vector
    from paper_2410_12614_amd import api

    m = config_mesh("c5")
    n_phi, n_q, q = 84, 512, 14
    u_h, v_h = normal_vector(m.n_dofs, 3), normal_vector(m.n_dofs, 4)
    out = {"workload": "P6 weighted stiffness action + VJP, 32^3 x 6 jittered Kuhn tetrahedra "
                       "(196,608 cells, 84 dofs/cell), 512-point rule, kappa interpolated in P6, "
                       "u, v ~ N(0,1)",
           "n_cells": m.n_cells, "n_dofs": m.n_dofs}
    res = {}
    for prec in ("fp32", "fp64"):
        dt = torch.float32 if prec == "fp32" else torch.float64
        mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs, m.coeff)
        act = api.Action(mv, api.form_desc(3, 6, q, "stiffness", prec, has_coeff=True))
        u = torch.from_numpy(u_h).to(dt).cuda()
        v = torch.from_numpy(v_h).to(dt).cuda()
        y = torch.empty_like(u)
        ms_fwd = time_steps(lambda: act.apply(u, out=y), steps, warmup)
        ms_vjp = time_steps(lambda: act.vjp(u, v), steps, warmup)
        gu, gz = act.vjp(u, v)
        torch.cuda.synchronize()
        if api.fe_get_device_status(act.form_buf) != 0:
            raise RuntimeError("device status after the action")
        res[prec] = {"ms_action": ms_fwd, "ms_vjp": ms_vjp, "y": y.double(), "gu": gu.double(),
                     "gz": gz.double()}
        del act, mv
    r32, r64 = res["fp32"], res["fp64"]
    err = {k: float(torch.linalg.vector_norm(r32[k] - r64[k]) / torch.linalg.vector_norm(r64[k]))
           for k in ("y", "gu", "gz")}
    ms = r32["ms_action"] + r32["ms_vjp"]
    # matrix-core work per cell (algorithmic, no padding): evaluation of
    # grad u (2 d n_q n_phi) and kappa (2 n_q n_phi) and the contraction
    # sum_s B_s r_s (2 d n_q n_phi) for the action; the VJP evaluates grad v,
    # grad u and kappa and contracts grad_u (d slabs) and grad_kappa (values)
    f_act = 2 * n_q * n_phi * (3 + 1 + 3)
    f_vjp = 2 * n_q * n_phi * (3 + 3 + 1 + 3 + 1)
    flops = (f_act + f_vjp) * m.n_cells
    ach = flops / (ms / 1e3) / 1e12
    out.update({
        "metric": "cells/s (action + VJP step)", "value": m.n_cells / (ms / 1e3),
        "unit": "cells/s", "dtype": "f32", "ms_per_step": ms,
        "ms_action": r32["ms_action"], "ms_vjp": r32["ms_vjp"],
        "fp64_path": {"value": m.n_cells / ((r64["ms_action"] + r64["ms_vjp"]) / 1e3),
                      "ms_action": r64["ms_action"], "ms_vjp": r64["ms_vjp"]},
        "rel_err_vs_fp64": err,
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_MFMA_TFLOPS["fp32"],
                     "unit": "TFLOP/s", "frac": ach / PEAK_MFMA_TFLOPS["fp32"], "traffic": None,
                     "kernel": "action_kernel + vector gather (both calls of the step)",
                     "alg_flops": flops},
    })
    del res
    if not args.no_cpu_baseline:
        n = m.n_cells if args.action_cpu_cells <= 0 else min(args.action_cpu_cells, m.n_cells)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        tab = oracle.tabulation(3, 6, q)
        uu, vv = u_h.astype(np.float64), v_h.astype(np.float64)
        t0 = time.perf_counter()
        b, _ = oracle.local_vectors("stiffness", m.cell_coords[:n], 6, q, m.dofmap[:n], uu,
                                    m.coeff, None, threads, tab)
        oracle.assemble_vector(m.dofmap[:n], b, m.n_dofs)
        b, g = oracle.local_vectors("stiffness", m.cell_coords[:n], 6, q, m.dofmap[:n], vv,
                                    m.coeff, uu, threads, tab)
        oracle.assemble_vector(m.dofmap[:n], b, m.n_dofs)
        oracle.assemble_vector(m.dofmap[:n], g, m.n_dofs)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": n / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} of {m.n_cells} cells (first n): action + VJP local vectors and "
                      f"vector assembly (FP64, {threads} OpenMP threads), one pass of {dt:.1f} s"}
    return out


def mixed_section(args, steps, warmup):
    """Mixed-degree batch: one graph launch for the eight degree blocks."""
    import numpy as np
    import torch

    import oracle
    from fe_inputs import mixed_degree_blocks
    from paper_2410_12614_amd import api

    blocks = mixed_degree_blocks()
    spec = [(b.degree, b.quad_degree, b.cell_coords, b.dofmap) for b in blocks]
    n_cells = sum(b.n_cells for b in blocks)
    out = {"workload": "mixed-degree DG mass, first 400,000 tets of 41^3 x 6 jittered Kuhn mesh, "
                       "p in 1..8 with P(p) ~ 1/p, quadrature degree 2p, one block per degree, "
                       "one block-diagonal CSR",
           "n_cells": n_cells, "cells_per_degree": {str(b.degree): b.n_cells for b in blocks}}
    md = api.MixedDegree(spec, "mass", "fp16")
    tuned = md.tune(reps=3)
    md.capture()
    ms = time_steps(md.numeric, steps, warmup)
    if any(st != 0 for st in md.status()):
        raise RuntimeError("device status after the mixed batch")
    v16 = md.numeric().clone()
    nnz = md.nnz
    out["tiles"] = {str(d): t for d, t, _ in tuned}
    del md
    torch.cuda.empty_cache()
    md64 = api.MixedDegree(spec, "mass", "fp64")
    md64.tune(reps=1)
    md64.capture()
    ms64 = time_steps(md64.numeric, max(3, steps // 2), max(1, warmup // 2))
    v64 = md64.numeric()
    torch.cuda.synchronize()
    err = float(torch.linalg.vector_norm(v16.double() - v64) / torch.linalg.vector_norm(v64))
    del md64, v64, v16
    torch.cuda.empty_cache()
    # algorithmic work: matrix-core flops 2 n_phi^2 n_q per cell, bytes = the
    # cells' coordinates read once and the values (4 B) written once
    flops = sum(b.n_cells * 2 * b.n_phi ** 2 * (b.degree + 1) ** 3 for b in blocks)
    nbytes = 96 * n_cells + 4 * nnz
    t = ms / 1e3
    ideal = {"hbm": nbytes / (PEAK_HBM_GBS * 1e9), "mfma": flops / (PEAK_MFMA_TFLOPS["fp16"] * 1e12)}
    bound = max(ideal, key=ideal.get)
    if bound == "hbm":
        roof = {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "mfma", "achieved": flops / t / 1e12, "peak": PEAK_MFMA_TFLOPS["fp16"],
                "unit": "TFLOP/s"}
    roof.update({"frac": roof["achieved"] / roof["peak"], "traffic": None,
                 "kernel": "cell_kernel per degree block (one graph launch)",
                 "ideal_us": {k: v * 1e6 for k, v in ideal.items()}, "alg_flops": flops,
                 "alg_bytes": nbytes})
    out.update({"metric": "cells/s (mixed-degree numeric phase, one graph launch)",
                "value": n_cells / t, "unit": "cells/s", "dtype": "f16 x f16 -> f32",
                "ms_per_step": ms, "nnz": nnz,
                "fp64_path": {"value": n_cells / (ms64 / 1e3), "ms_per_step": ms64},
                "speedup_vs_fp64": ms64 / ms, "rel_err_vs_fp64": err, "roofline": roof})
    if not args.no_cpu_baseline:
        n = min(args.mixed_cpu_cells, n_cells)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        t0 = time.perf_counter()
        for b in blocks:
            sel = b.cell_ids < n       # the first n cells of the source mesh
            if sel.any():
                oracle.local_matrices("mass", b.cell_coords[sel], b.degree, b.quad_degree,
                                      nthreads=threads)
        dt = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": n / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of {n_cells} cells (all degrees, same mix): local matrices "
                      f"(FP64, {threads} OpenMP threads; the block-diagonal assembly is the "
                      f"local matrices themselves), one pass of {dt:.1f} s"}
    return out


def hex_section(args, steps, warmup, form="mass"):
    """A form on trilinear hexahedra (Q4): FE_NUMERIC in FP16 and FP64."""
    import numpy as np
    import torch

    from fe_inputs import hex_mesh
    from paper_2410_12614_amd import _lib as L
    from paper_2410_12614_amd import api

    m = hex_mesh(38, 4, jitter=0.25, seed=0)
    n_cells, n_phi, n_q = m.cell_coords.shape[0], 125, 125
    nd = 1 if form == "mass" else 3
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs)
    what = "|det J| per point" if form == "mass" else "G = |det J| J^-1 J^-T per point"
    out = {"workload": f"Q4 {form} on 38^3 jittered trilinear hexahedra (54,872 cells, 125 dofs/cell), "
                       f"125-point tensor Gauss-Legendre rule, {what}",
           "n_cells": n_cells, "n_dofs": m.n_dofs}
    res = {}
    for prec in ("fp16", "fp64"):
        log(f"hexahedral {form}: {prec}")
        asm = api.Assembly(mv, [api.form_desc(L.FE_HEXAHEDRON, 4, 8, form, prec)])
        res[prec] = time_steps(asm.numeric, steps if prec == "fp16" else max(3, steps // 2), warmup)
        if prec == "fp16":
            if form == "mass":
                # the cell kernels + row gather, for comparison
                res["gather"] = time_steps(lambda: asm.numeric(gather=True), max(3, steps // 2), warmup)
            else:
                res["local"] = time_steps(lambda: asm.numeric(part="local"), max(3, steps // 2), warmup)
                res["assemble"] = time_steps(lambda: asm.numeric(part="assemble"), max(3, steps // 2),
                                             warmup)
        if any(st != 0 for st in asm.status()):
            raise RuntimeError("device status after the hexahedral step")
        res[prec + "_vals"] = asm.numeric()[0][:asm.nnz].double().clone()
        nnz = asm.nnz
        del asm
        torch.cuda.empty_cache()
    err = float(torch.linalg.vector_norm(res["fp16_vals"] - res["fp64_vals"]) /
                torch.linalg.vector_norm(res["fp64_vals"]))
    del res["fp16_vals"], res["fp64_vals"]
    ms = res["fp16"]
    flops = n_cells * 2 * n_phi ** 2 * nd * n_q
    nbytes = (192 + 4 * n_phi) * n_cells + 4 * nnz
    t = ms / 1e3
    ideal = {"hbm": nbytes / (PEAK_HBM_GBS * 1e9), "mfma": flops / (PEAK_MFMA_TFLOPS["fp16"] * 1e12)}
    if max(ideal, key=ideal.get) == "hbm":
        roof = {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
    else:
        roof = {"bound": "mfma", "achieved": flops / t / 1e12, "peak": PEAK_MFMA_TFLOPS["fp16"],
                "unit": "TFLOP/s"}
    roof.update({"frac": roof["achieved"] / roof["peak"], "traffic": None,
                 "kernel": ("k_box_geo + fused row-ownership pass (the whole step)" if form == "mass"
                            else "cell kernels with per-point G + row gather (the whole step)"),
                 "ideal_us": {k: v * 1e6 for k, v in ideal.items()}, "alg_flops": flops,
                 "alg_bytes": nbytes})
    out.update({"metric": f"cells/s (hexahedral {form}, kernels + CSR assembly)",
                "value": n_cells / t, "unit": "cells/s", "dtype": "f16 x f16 -> f32",
                "ms_per_step": ms, "nnz": nnz,
                "fp64_path": {"value": n_cells / (res["fp64"] / 1e3), "ms_per_step": res["fp64"]},
                "speedup_vs_fp64": res["fp64"] / ms, "rel_err_vs_fp64": err, "roofline": roof})
    if form == "mass":
        out["gather_path_fp16_ms"] = res["gather"]
    else:
        out["kernels"] = {"local_matrices": {"ms": res["local"]}, "row_gather": {"ms": res["assemble"]}}
    if not args.no_cpu_baseline:
        import oracle
        import oracle.hexahedra as H
        log(f"hexahedral {form}: oracle baseline")
        n = min(args.hex_cpu_cells if form == "mass" else args.hex_cpu_cells // 3, n_cells)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        rp, ci = oracle.csr_pattern(m.dofmap[:n], m.n_dofs)      # symbolic: not timed
        t0 = time.perf_counter()
        A = H.local_matrices(form, m.cell_coords[:n], 4, 8, nthreads=threads)
        oracle.assemble(m.dofmap[:n], A, m.n_dofs, rp, ci)
        dt = time.perf_counter() - t0
        del A
        n1 = min(1000 if form == "mass" else 300, n)
        rp1, ci1 = oracle.csr_pattern(m.dofmap[:n1], m.n_dofs)
        t0 = time.perf_counter()
        A = H.local_matrices(form, m.cell_coords[:n1], 4, 8, nthreads=1)
        oracle.assemble(m.dofmap[:n1], A, m.n_dofs, rp1, ci1)
        dt1 = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": n / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of {n_cells} cells: local {form} matrices (FP64, per-point "
                      f"geometry, {threads} OpenMP threads) + CSR assembly, one pass of {dt:.1f} s",
            "single_thread": {"value": n1 / dt1, "unit": "cells/s", "cores": 1,
                              "sample": f"first {n1} cells, one pass of {dt1:.1f} s"}}
    return out


def c3_section(args, steps, warmup):
    """Weighted P6 stiffness (the coefficient workload) in BF16, FP16, FP32
    and FP64: FE_NUMERIC (cell kernels + CSR assembly), each mode's cell
    kernel timed alone for its matrix-core roofline, relative Frobenius error
    of every mode against the FP64 result, and an oracle baseline sample."""
    import numpy as np
    import torch

    from fe_inputs import config_mesh
    from paper_2410_12614_amd import api

    m = config_mesh("c3")
    n_phi, n_q, q = 84, 512, 14
    mv = api.MeshView.from_numpy(m.cell_coords, m.dofmap, m.n_dofs, m.coeff)
    # algorithmic matrix-core work per cell: the contraction 2 n_phi^2 (d n_q)
    # and the coefficient at the points 2 n_phi n_q (no padding counted)
    f_con = 2 * n_phi ** 2 * 3 * n_q
    f_coef = 2 * n_phi * n_q
    flops = (f_con + f_coef) * m.n_cells
    # what the FP16 whole-cell kernel executes on the matrix cores: the 21
    # tiles (I <= J) of the 6 x 6 row-tile grid (padded to 96), K = 3 n_q,
    # plus the coefficient pass (n_q x 96 x 16-cell tiles)
    hw_flops = (21 * 2 * 16 * 16 * 3 * n_q + 2 * n_q * 96) * m.n_cells
    out = {"workload": "P6 weighted stiffness div(kappa grad u), 32^3 x 6 jittered Kuhn tetrahedra "
                       "(196,608 cells, 84 dofs/cell), 512-point collapsed Gauss-Jacobi rule, "
                       "kappa = exp(sin(2 pi x) cos(2 pi y) z) interpolated in P6, FP64 geometry",
           "n_cells": m.n_cells, "n_dofs": m.n_dofs, "alg_flops": flops,
           "alg_flops_per_cell": {"contraction": f_con, "coefficient": f_coef}}
    modes, vals = {}, {}
    # FP64 first: its values are the reference of the other modes' errors
    for prec in ("fp64", "fp32", "bf16", "fp16"):
        log(f"weighted P6 stiffness: {prec}")
        desc = api.form_desc(3, 6, q, "stiffness", prec, has_coeff=True)
        asm = api.Assembly(mv, [desc])
        k = steps if prec in ("fp16", "bf16") else max(3, steps // 4)
        w = warmup if prec in ("fp16", "bf16") else max(1, warmup // 2)
        ms = time_steps(asm.numeric, k, w)
        # the two halves of the step: local matrices (for FP16 the
        # coefficient at the points, then the whole-cell kernel), row gather
        ms_cell = time_steps(lambda: asm.numeric(part="local"), k, w)
        ms_gather = time_steps(lambda: asm.numeric(part="assemble"), k, w)
        (v,) = asm.numeric()
        torch.cuda.synchronize()
        if any(st != 0 for st in asm.status()):
            raise RuntimeError(f"device status after the weighted-stiffness step ({prec})")
        nnz = asm.nnz
        vals[prec] = v[:nnz].clone()
        peak = PEAK_MFMA_TFLOPS[prec]
        t_cell = ms_cell / 1e3
        modes[prec] = {
            "ms_per_step": ms, "value": m.n_cells / (ms / 1e3), "unit": "cells/s",
            "dtype": {"fp16": "f16 x f16 -> f32", "bf16": "bf16 x bf16 -> f32", "fp32": "f32",
                      "fp64": "f64"}[prec],
            "kernels": {"local_matrices": {"ms": ms_cell}, "row_gather": {"ms": ms_gather}},
            "roofline": {"bound": "mfma", "achieved": flops / t_cell / 1e12, "peak": peak,
                         "unit": "TFLOP/s", "frac": flops / t_cell / 1e12 / peak, "traffic": None,
                         "kernel": ("coefficient at the points + whole-cell kernel (a2-a5 of every "
                                    "cell)" if prec == "fp16" else "cell_kernel (a2-a5 of every cell)"),
                         "step_frac": flops / (ms / 1e3) / 1e12 / peak},
        }
        del asm
        torch.cuda.empty_cache()
    ref = vals["fp64"]
    nref = float(torch.linalg.vector_norm(ref))
    for prec in ("fp32", "bf16", "fp16"):
        err = float(torch.linalg.vector_norm(vals[prec].double() - ref)) / nref
        modes[prec]["rel_err_vs_fp64"] = err
        modes[prec]["speedup_vs_fp64"] = modes["fp64"]["ms_per_step"] / modes[prec]["ms_per_step"]
    del vals, ref
    torch.cuda.empty_cache()
    out["nnz"] = nnz
    out["modes"] = modes
    f16 = modes["fp16"]
    t16 = f16["kernels"]["local_matrices"]["ms"] / 1e3
    f16["roofline"]["mfma_executed_tflops"] = hw_flops / t16 / 1e12
    f16["roofline"]["mfma_executed_frac"] = hw_flops / t16 / 1e12 / PEAK_MFMA_TFLOPS["fp16"]
    # HBM bytes of the whole-cell kernel and of the row gather (measured,
    # per launch); the gather is bound by HBM
    f16["roofline"]["traffic"] = measured_traffic(CW_TRAFFIC_FILE, CW_SOURCES)
    gb = measured_traffic(GATHER_TRAFFIC_FILE, GATHER_SOURCES)
    if gb is not None:
        tg = f16["kernels"]["row_gather"]["ms"] / 1e3
        f16["kernels"]["row_gather"].update({"traffic": gb, "gbs": gb / tg / 1e9,
                                            "frac_hbm": gb / tg / 1e9 / PEAK_HBM_GBS})
    out.update({"metric": "cells/s (weighted P6 stiffness, kernels + CSR assembly)",
                "value": f16["value"], "unit": "cells/s", "dtype": f16["dtype"],
                "ms_per_step": f16["ms_per_step"], "roofline": f16["roofline"],
                "rel_err_vs_fp64": f16["rel_err_vs_fp64"],
                "speedup_vs_fp64": f16["speedup_vs_fp64"]})
    if not args.no_cpu_baseline:
        import oracle
        log("weighted P6 stiffness: oracle baseline")
        n = min(args.c3_cpu_cells, m.n_cells)
        threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or (os.cpu_count() or 1)
        tab = oracle.tabulation(3, 6, q)
        rp, ci = oracle.csr_pattern(m.dofmap[:n], m.n_dofs)      # symbolic: not timed
        t0 = time.perf_counter()
        A = oracle.local_matrices("stiffness", m.cell_coords[:n], 6, q, m.dofmap[:n], m.coeff,
                                  nthreads=threads, tab=tab)
        oracle.assemble(m.dofmap[:n], A, m.n_dofs, rp, ci)
        dt = time.perf_counter() - t0
        del A
        n1 = min(256, n)
        rp1, ci1 = oracle.csr_pattern(m.dofmap[:n1], m.n_dofs)
        t0 = time.perf_counter()
        A = oracle.local_matrices("stiffness", m.cell_coords[:n1], 6, q, m.dofmap[:n1], m.coeff,
                                  nthreads=1, tab=tab)
        oracle.assemble(m.dofmap[:n1], A, m.n_dofs, rp1, ci1)
        dt1 = time.perf_counter() - t0
        out["cpu_baseline"] = {
            "value": n / dt, "unit": "cells/s", "cores": threads, "kind": "oracle",
            "sample": f"first {n} of {m.n_cells} cells: local matrices (coefficient at the points, "
                      f"FP64) + CSR assembly, {threads} OpenMP threads, one pass of {dt:.1f} s",
            "single_thread": {"value": n1 / dt1, "unit": "cells/s", "cores": 1,
                              "sample": f"first {n1} cells, one pass of {dt1:.1f} s"}}
    return out


def sources_digest(sources=None):
    """SHA-256 over a kernel's sources (traffic is reported only for the
    code it was measured on)."""
    import hashlib
    h = hashlib.sha256()
    for f in sources or KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2410_12614_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path=TRAFFIC_FILE, sources=None):
    """Fetch + write bytes per launch of a kernel from its committed counter
    summary, or None when absent or measured on other code."""
    if not os.path.exists(path):
        return None
    vals = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            vals[k.strip()] = v.strip()
    if vals.get("sources_sha256") != sources_digest(sources):
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU only (asked for --gpus {args.gpus}); "
              "sharding over several GPUs is designed, not implemented", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from fe_inputs import config_mesh
    from paper_2410_12614_amd import _lib as L
    from paper_2410_12614_amd import api

    mesh = config_mesh("c2")
    mv = api.MeshView.from_numpy(mesh.cell_coords, mesh.dofmap, mesh.n_dofs)
    forms = ("mass", "stiffness")

    def assembly(prec):
        return api.Assembly(mv, [api.form_desc(3, 4, 8, f, prec) for f in forms])

    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device="cuda")   # 256 MiB
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    prec = args.precision
    n_phi = mesh.n_phi
    n_q = 125
    kq = {"mass": n_q, "stiffness": 3 * n_q}
    flops = sum(2 * n_phi ** 2 * kq[f] * mesh.n_cells for f in forms)

    # Roofline of the dominant kernel: the fused pass (both forms).  Its
    # algorithmic work per launch: matrix-core flops 2 n_phi^2 K per cell and
    # form (K = n_q mass, 3 n_q stiffness); H formation d^2 n_q n_phi FMAs per
    # cell for stiffness, n_q n_phi for mass; bytes: each cell's coordinates
    # (96) and dof map (4 n_phi) read once, each form's CSR values (4 nnz)
    # written once.
    valu = sum(2 * (9 if f == "stiffness" else 1) * n_q * n_phi * mesh.n_cells for f in forms)

    def c2_roofline(pr, t, nnz):
        nbytes = (96 + 4 * n_phi) * mesh.n_cells + len(forms) * 4 * nnz
        ideal = {"hbm": nbytes / (PEAK_HBM_GBS * 1e9),
                 "mfma": flops / (PEAK_MFMA_TFLOPS[pr] * 1e12),
                 "alu": valu / (PEAK_VALU_TFLOPS * 1e12)}
        bound = max(ideal, key=ideal.get)
        if bound == "hbm":
            roof = {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM_GBS, "unit": "GB/s"}
        elif bound == "mfma":
            roof = {"bound": "mfma", "achieved": flops / t / 1e12, "peak": PEAK_MFMA_TFLOPS[pr],
                    "unit": "TFLOP/s"}
        else:
            roof = {"bound": "alu", "achieved": valu / t / 1e12, "peak": PEAK_VALU_TFLOPS,
                    "unit": "TFLOP/s"}
        roof["frac"] = roof["achieved"] / roof["peak"]
        roof["kernel"] = "fused_pass"
        roof["ideal_us"] = {k: v * 1e6 for k, v in ideal.items()}
        roof["alg_bytes"] = nbytes
        return roof

    # The FP64 path and the other mixed modes first (their values are kept
    # for the error of each mode against FP64), then the reported mode.
    result, v64, other = {}, None, {}
    log("P4 mass+stiffness: FP64 path")
    if not args.no_fp64:
        asm64 = assembly("fp64")
        ms64 = time_steps(asm64.numeric, max(3, args.steps // 4), max(1, args.warmup // 5))
        v64 = [v[:asm64.nnz].clone() for v in asm64.numeric()]
        torch.cuda.synchronize()
        result["fp64_path"] = {"value": mesh.n_cells / (ms64 / 1e3), "ms_per_step": ms64}
        del asm64
        torch.cuda.empty_cache()

    def rel_errs(vals, nnz):
        return {f: float(torch.linalg.vector_norm(a[:nnz].double() - b) / torch.linalg.vector_norm(b))
                for f, a, b in zip(forms, vals, v64)}

    for other_prec in ("split", "bf16"):
        if other_prec == prec:
            continue
        log(f"P4 mass+stiffness: {other_prec}")
        a2 = assembly(other_prec)
        ms2 = time_steps(a2.numeric, args.steps, args.warmup)
        try:
            # the fused pass alone, where every form of the pair takes it
            ms2_fused = time_steps(lambda: a2.numeric(part="fused"), args.steps, args.warmup)
            roof_kernel = "fused_pass"
        except L.FeError:
            ms2_fused = ms2
            roof_kernel = "whole step (cell kernels + row gather for a form off the fused path)"
        if any(st != 0 for st in a2.status()):
            raise RuntimeError(f"device status ({other_prec})")
        roof2 = c2_roofline(other_prec, ms2_fused / 1e3, a2.nnz)
        roof2["kernel"] = roof_kernel
        roof2["traffic"] = None
        other[other_prec] = {
            "ms_per_step": ms2, "value": mesh.n_cells / (ms2 / 1e3), "unit": "cells/s",
            "dtype": {"bf16": "bf16 x bf16 -> f32", "split": "2xf16 x 2xf16 -> f32"}[other_prec],
            "roofline_ms": ms2_fused, "roofline": roof2,
        }
        if v64 is not None:
            other[other_prec]["rel_err_vs_fp64"] = rel_errs(a2.numeric(), a2.nnz)
            other[other_prec]["speedup_vs_fp64"] = result["fp64_path"]["ms_per_step"] / ms2
        del a2
        torch.cuda.empty_cache()

    log(f"P4 mass+stiffness: {prec} (reported)")
    asm = assembly(prec)
    ms = time_steps(asm.numeric, args.steps, args.warmup)
    st = asm.status()
    if any(s != 0 for s in st):
        raise RuntimeError(f"device status {st}")

    # the two halves of the step, and the unfused path for comparison
    nnz = asm.nnz
    ms_geo = time_steps(lambda: asm.numeric(part="geometry"), args.steps, args.warmup)
    ms_fused = time_steps(lambda: asm.numeric(part="fused"), args.steps, args.warmup)
    ms_gather_path = time_steps(lambda: asm.numeric(gather=True), max(3, args.steps // 4),
                                max(1, args.warmup // 5))
    if v64 is not None:
        result["speedup_vs_fp64"] = result["fp64_path"]["ms_per_step"] / ms
        result["rel_err_vs_fp64"] = rel_errs(asm.numeric(), nnz)
    if other:
        result["other_modes"] = other
    del v64

    t = ms_fused / 1e3
    roof = c2_roofline(prec, t, nnz)
    nbytes = roof["alg_bytes"]
    kern = {"fused_pass": {"ms": ms_fused, "alg_flops": flops, "alg_valu_flops": valu,
                           "alg_bytes": nbytes, "tflops": flops / t / 1e12,
                           "gbs": nbytes / t / 1e9},
            "geometry_pass": {"ms": ms_geo},
            "unfused_step": {"ms": ms_gather_path}}
    roof["traffic"] = measured_traffic() if prec == "fp16" else None

    line = {
        "metric": "cells/sec (kernel+CSR assembly) mixed FP16/FP32 vs FP64 at stated rel. error",
        "value": mesh.n_cells / (ms / 1e3),
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp16": "f16 x f16 -> f32", "bf16": "bf16 x bf16 -> f32",
                  "split": "2xf16 x 2xf16 -> f32", "fp32": "f32"}[prec],
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n_cells": mesh.n_cells, "degree": 4, "quad_degree": 8,
                   "forms": list(forms), "precision": prec, "geometry": "f64", "nnz": nnz,
                   "n_dofs": mesh.n_dofs, "assembly": "fused row ownership"},
        "roofline": roof,
        "kernels": kern,
        **result,
    }
    if not args.no_cpu_baseline:
        log("P4 mass+stiffness: oracle baseline")
        line["cpu_baseline"] = cpu_baseline(mesh, args.cpu_sample_cells, args.cpu_reps)
    del asm
    torch.cuda.empty_cache()
    if not args.no_action:
        log("action + VJP")
        line["action_vjp"] = action_section(args, max(3, args.steps // 2), max(1, args.warmup // 5))
    if not args.no_mixed:
        torch.cuda.empty_cache()
        log("mixed-degree batch")
        line["mixed_degree"] = mixed_section(args, max(3, args.steps // 4), max(1, args.warmup // 5))
    if not args.no_hex:
        torch.cuda.empty_cache()
        line["hex_mass"] = hex_section(args, max(3, args.steps // 4), max(1, args.warmup // 5))
        torch.cuda.empty_cache()
        line["hex_stiffness"] = hex_section(args, max(3, args.steps // 4), max(1, args.warmup // 5),
                                            form="stiffness")
    if not args.no_c3:
        torch.cuda.empty_cache()
        log("weighted P6 stiffness")
        line["weighted_p6"] = c3_section(args, max(3, args.steps // 4), max(1, args.warmup // 5))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
