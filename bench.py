#!/usr/bin/env python3
"""Benchmark: column-generation VMAT iterations on one MI355X.

One step = one column-generation iteration of Sec. 2.1 on the full-scale
single-arc workload (180 control points x 40x40 beamlets of 5 mm, 128^3
voxels of 2.5 mm, ~5e8 non-zeros): price-based aperture selection, adding the
aperture, then a 50-iteration Barzilai-Borwein master-problem solve, each
iteration a dose product with the fused objective and a price product over
the whole DDC matrix, plus one curvature product for the first step length.

Output: one JSON line on stdout.  `value` is the HBM bandwidth of the whole
timed job (algorithmic bytes of every product / wall time, inputs resident in
HBM), `ms_per_step` the time per column-generation iteration.  Algorithmic
bytes count the matrix with the index width of its own layout (2-byte
panel-local columns, 4-byte CSR columns, one index per B rows of a block row);
`csr_equivalent_gbs` is the same time over the bytes of FP32/16-bit values
with int32 CSR indices, the usual "effective" figure.  Progress goes to stderr.

    python bench.py [--steps K] [--warmup W] [--storage f32|f16|bf16]

Other modes, each printing its own JSON line: --form DA (the paper's DA form
of the master problem), --mode batched (many plans x 8 right-hand sides in
one captured launch against one plan at a time), --mode autograd (F(D B y)
and dF/dy by automatic differentiation on the two-arc workload), --mode shard
(one GPU's voxel slab of the two-arc workload at its real shape), --mode
truncation (plans optimised on cone-truncated matrices, Sec. 2.4 S1,
re-evaluated on the complete matrix).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

METRIC = "effective HBM GB/s (and % peak) for D·x + Dᵀ·g; ms per column-gen iteration"
HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def index_bytes(info, orientation):
    """Index bytes per stored non-zero of one orientation as built: 2 for the
    panel layout's panel-local uint16 columns, 4 for CSR's int32 columns, shared
    by the B rows of a block row (one index per stored position serves B rows).
    Padding zeros of block rows and the panels' column lists are format
    overhead and not counted."""
    layout = info.dose_layout if orientation == "dose" else info.price_layout
    B = max(1, info.dose_block_rows if orientation == "dose" else info.price_block_rows)
    return (2.0 if layout >= 1 else 4.0) / B


LAYOUT_NAMES = {0: "csr", 1: "panel", 2: "sliced"}
KERNEL_NAMES = {0: "spmv_kernel", 1: "spmv_panel_kernel", 2: "spmv_slice_kernel"}


def grid_layout(args, grids):
    """Build options of --layout: CSR, or the grids with the library's default
    grid layout (sliced panels), or panels / sliced panels forced."""
    if args.layout == "csr":
        return {}
    out = dict(grids)
    if args.layout in ("panel", "sliced"):
        out.update(dose_layout=args.layout, price_layout=args.layout)
    if args.layout != "panel":
        if args.dose_lanes:
            out["dose_slice_lanes"] = args.dose_lanes
        if args.price_lanes:
            out["price_slice_lanes"] = args.price_lanes
    return out


def algorithmic_bytes(info, nrhs=1, csr_equivalent=False):
    """Bytes each product must move: the matrix once (values plus the layout's
    own index bytes, or 4-byte indices for the CSR-equivalent figure), row
    pointers, each vector once, the objective's per-voxel inputs and outputs,
    the per-beamlet scale at 16-bit storage."""
    n_vox, n_bl, nnz = info.n_vox, info.n_bl, info.nnz
    ib_d = 4.0 if csr_equivalent else index_bytes(info, "dose")
    ib_p = 4.0 if csr_equivalent else index_bytes(info, "price")
    mat_d = int(round(nnz * (info.value_bytes + ib_d)))
    mat_p = int(round(nnz * (info.value_bytes + ib_p)))
    scale = 4 * n_bl if info.value_bytes == 2 else 0
    dose_obj = mat_d + 8 * (n_vox + 1) + 4 * nrhs * (n_bl + n_vox) + n_vox * (1 + 4 * nrhs) + scale
    price = mat_p + 8 * (n_bl + 1) + 4 * nrhs * (n_vox + n_bl) + scale
    curv = mat_d + 8 * (n_vox + 1) + 4 * n_bl + n_vox * (4 + 1) + scale
    return dict(dose=dose_obj, price=price, curv=curv)


def read_traffic(kernel, workload, storage, layout):
    """HBM traffic per launch from the committed counter summary, if it was taken
    on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{storage}_{layout}.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if "=" in line and not line.startswith("#"):
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    from paper_1503_01721_amd.profiling import products_source_sha
    if kv.get("products_source_sha256_16") != products_source_sha():
        return None
    try:
        return float(kv["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def cpu_baseline(d, plan, bytes_dose_plain, bytes_price, min_seconds=10.0, max_pairs=6):
    """The FP64 oracle (NumPy bincount over COO, single-threaded) on pairs of one
    dose and one price product over the whole matrix, repeated until at least
    min_seconds of CPU work (at most max_pairs pairs)."""
    import numpy as np
    from oracle import products as oprod
    from paper_1503_01721_amd import synth
    x, g = synth.bench_vectors(plan.n_bl, plan.n_vox, 1002)
    t_dose = t_price = 0.0
    pairs = 0
    while pairs < max_pairs and (pairs == 0 or t_dose + t_price < min_seconds):
        t0 = time.perf_counter()
        oprod.dose(d["row"], d["col"], d["val"], x, plan.n_vox)
        t1 = time.perf_counter()
        oprod.price(d["row"], d["col"], d["val"], g, plan.n_bl)
        t2 = time.perf_counter()
        t_dose += t1 - t0
        t_price += t2 - t1
        pairs += 1
    gbs = pairs * (bytes_dose_plain + bytes_price) / (t_dose + t_price) / 1e9
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(line.split(":", 1)[1].strip() for line in fh if line.startswith("model name"))
    except (OSError, StopIteration):
        pass
    affinity = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": round(gbs, 3), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": (f"{pairs} pair{'s' if pairs != 1 else ''} of one FP64 dose and one FP64 price product over the whole {plan.name} "
                       f"matrix (NumPy bincount over COO, single-threaded; dose {t_dose / pairs:.2f} s, "
                       f"price {t_price / pairs:.2f} s per product); "
                       f"host {model}, os.cpu_count()={os.cpu_count()}, affinity {affinity} CPUs"),
            "seconds": round(t_dose + t_price, 3)}


def copy_calibration():
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    n = 1 << 28                                     # 1 GiB of float32
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(5):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": 4 * n, "copy_calibration_bytes_written": 4 * n,
                      "launches": 5}), flush=True)


def plain_bytes(info, nrhs, csr_equivalent=False):
    """Algorithmic bytes of a plain dose and a plain price product with nrhs vectors."""
    n_vox, n_bl, nnz = info.n_vox, info.n_bl, info.nnz
    ib_d = 4.0 if csr_equivalent else index_bytes(info, "dose")
    ib_p = 4.0 if csr_equivalent else index_bytes(info, "price")
    scale = 4 * n_bl if info.value_bytes == 2 else 0
    return (int(round(nnz * (info.value_bytes + ib_d))) + 8 * (n_vox + 1) + 4 * nrhs * (n_bl + n_vox) + scale,
            int(round(nnz * (info.value_bytes + ib_p))) + 8 * (n_bl + 1) + 4 * nrhs * (n_vox + n_bl) + scale)


def check_peak(name, gbs):
    """A rate above the HBM peak means the byte count is wrong, not a fast kernel."""
    if gbs > HBM_PEAK_GBS:
        log(f"WARNING: {name} at {gbs:.0f} GB/s exceeds the {HBM_PEAK_GBS:.0f} GB/s HBM peak: "
            "its algorithmic bytes overcount what it moves")
    return gbs <= HBM_PEAK_GBS


def bench_batched(args):
    """Many plans of uneven size, 8 right-hand sides each: one captured graph of
    the batched dose and price launches vs one launch per plan."""
    import torch
    from paper_1503_01721_amd import dvmat, synth
    storage = args.storage if args.storage != "f32" or "--storage" in sys.argv else "f16"
    plans = synth.batched_plans(args.plans, 2005)
    nrhs = 8
    ddcs, t_gen, t_build = [], 0.0, 0.0
    for i, p in enumerate(plans):
        t = time.perf_counter()
        d = synth.generate_ddc(p)
        t_gen += time.perf_counter() - t
        t = time.perf_counter()
        # multi-vector panels pay where a slice serves many rows: the dose (a
        # voxel tile touches few beamlets); a beamlet row alone touches ~2000
        # voxels, so the price stays in CSR
        layout = {} if args.layout == "csr" else dict(panel_cols=args.panel_cols, dose_layout=args.batch_dose_layout,
                                                       price_layout=args.batch_price_layout, **p.grids)
        if args.layout != "csr" and args.batch_dose_layout == "panel":
            layout["dose_block_rows"] = args.batch_dose_b
        # the plans of a batch share their lanes per row (the library would
        # choose them per plan from the rows' lengths)
        if args.layout != "csr":
            # 16 lanes: a 16-lane pass of the 16-byte gathers of 4 right-hand
            # sides then reads one row's neighbouring columns (fewer LDS bank
            # conflicts; 16 plans: 14.3 ms against 15.1 with 4)
            layout["dose_slice_lanes"] = args.dose_lanes or 16
            layout["price_slice_lanes"] = args.price_lanes or 8
        if args.batch_price_b and args.batch_price_layout != "sliced":
            layout["price_block_rows"] = args.batch_price_b
        ddcs.append(dvmat.DDC(d["row"], d["col"], d["val"], p.n_vox, p.n_bl, storage=storage, **layout))
        t_build += time.perf_counter() - t
        del d
        if i % 8 == 7 or i == len(plans) - 1:
            log(f"built {i + 1}/{len(plans)} plans (generate {t_gen:.1f} s, build {t_build:.1f} s)")
    nnz = sum(x.info.nnz for x in ddcs)
    gen = torch.Generator(device="cuda").manual_seed(2005)
    X = [torch.rand((x.n_bl, nrhs), device="cuda", generator=gen) for x in ddcs]
    G = [torch.randn((x.n_vox, nrhs), device="cuda", generator=gen) for x in ddcs]
    Z = [torch.empty((x.n_vox, nrhs), device="cuda") for x in ddcs]
    P = [torch.empty((x.n_bl, nrhs), device="cuda") for x in ddcs]
    batch = dvmat.Batch(ddcs)
    if not args.no_autotune:
        binfo = batch.autotune(X, Z, G, P, reps=3)
        for x in ddcs:
            x.autotune(reps=3)
        log(f"autotuned: batch {binfo}")
    binfo = batch.info()
    total = sum(sum(plain_bytes(x.info, nrhs)) for x in ddcs)
    total_csr = sum(sum(plain_bytes(x.info, nrhs, csr_equivalent=True)) for x in ddcs)
    # batched: one captured graph holding the two launches
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        batch.dose_(X, Z)
        batch.price_(G, P)
        s.synchronize()
        with torch.cuda.graph(graph, stream=s):
            batch.dose_(X, Z)
            batch.price_(G, P)
    torch.cuda.current_stream().wait_stream(s)
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        graph.replay()
    torch.cuda.synchronize()
    t_batched = (time.perf_counter() - t0) / args.steps
    # one plan at a time
    for _ in range(args.warmup):
        for x, xx, zz, gg, pp in zip(ddcs, X, Z, G, P):
            x.dose_(xx, zz)
            x.price_(gg, pp)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for x, xx, zz, gg, pp in zip(ddcs, X, Z, G, P):
            x.dose_(xx, zz)
            x.price_(gg, pp)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / args.steps
    gbs_b, gbs_s = total / t_batched / 1e9, total / t_seq / 1e9
    check_peak("batched step", gbs_b)
    log(f"batched {t_batched * 1e3:.2f} ms ({gbs_b:.0f} GB/s) vs one-plan-at-a-time {t_seq * 1e3:.2f} ms "
        f"({gbs_s:.0f} GB/s)")
    print(json.dumps({
        "metric": "aggregate effective HBM GB/s of dose + price over all plans (batched launch)",
        "value": round(gbs_b, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(t_batched * 1e3, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": storage, "data": "synthetic",
        "config": {"workload": f"{len(plans)} uneven plans x {nrhs} right-hand sides", "nnz_total": int(nnz),
                   "layout": args.layout if args.layout == "csr" else
                   f"{args.batch_dose_layout} (dose), {args.batch_price_layout} (price)",
                   "dose_block_rows": args.batch_dose_b if args.batch_dose_layout == "panel" else 1,
                   "panel_cols": args.panel_cols,
                   "storage": storage, "nrhs": nrhs, "algorithmic_bytes_per_step": int(total),
                   "csr_equivalent_gbs": round(total_csr / t_batched / 1e9, 2),
                   "one_plan_at_a_time_gbs": round(gbs_s, 2), "one_plan_at_a_time_ms": round(t_seq * 1e3, 3),
                   "speedup_vs_one_plan_at_a_time": round(t_seq / t_batched, 3),
                   "pct_hbm_peak": round(100.0 * gbs_b / HBM_PEAK_GBS, 2), "batch_launch": binfo,
                   "generate_s": round(t_gen, 1), "build_upload_s": round(t_build, 1)},
    }), flush=True)


def bench_autograd(args):
    """Differentiation form: F(D B y) and dF/dy by autograd (dose forward, price
    backward) for 64 random apertures on the two-arc workload."""
    import numpy as np
    import torch
    from paper_1503_01721_amd import dvmat, synth
    from paper_1503_01721_amd.autograd import plan_objective
    workload = args.workload if args.workload != "cp180_bl40x40_vox128" else "cp360_bl60x60_vox160"
    storage = args.storage if "--storage" in sys.argv else "f16"
    plan = synth.PLANS[workload]
    t = time.perf_counter()
    d = synth.generate_ddc(plan)
    sid, table = synth.structures(plan)
    t_gen = time.perf_counter() - t
    log(f"generated {plan.name}: nnz={len(d['val'])} in {t_gen:.1f} s")
    t = time.perf_counter()
    layout = grid_layout(args, plan.grids)
    ddc = dvmat.DDC(d["row"], d["col"], d["val"], plan.n_vox, plan.n_bl, storage=storage, **layout)
    del d
    obj = dvmat.Objective(sid, table)
    t_build = time.perf_counter() - t
    log(f"built and uploaded {ddc.info.workspace_bytes / 2**30:.1f} GiB in {t_build:.1f} s")
    if not args.no_autotune:
        ddc.autotune(reps=3)
    cps, L, R = synth.random_apertures(plan, 64, 2004)
    aps = dvmat.Apertures(plan.n_cp, plan.n_rows, plan.n_cols, cps, L, R)
    # rates scaled so that the mean PTV dose is the prescription at y = 1
    x1 = torch.empty(plan.n_bl, device="cuda")
    aps.expand_(torch.ones(64, device="cuda"), x1)
    z1 = ddc.dose(x1)
    ptv = torch.from_numpy(sid == synth.S_PTV0).cuda()
    scale = 70.0 / float(z1[ptv].mean())
    rng = np.random.default_rng(2004)
    y = torch.tensor(rng.uniform(0.5, 1.5, 64) * scale, dtype=torch.float32, device="cuda", requires_grad=True)

    def step():
        y.grad = None
        F = plan_objective(y, aps, ddc, obj)
        F.backward()
        return F

    for _ in range(max(args.warmup, 1)):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        F = step()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    bd, bp = plain_bytes(ddc.info, 1)
    extra = plan.n_vox * (4 + 1 + 4) + 4 * plan.n_bl            # objective pass, fluence expansion
    gbs = (bd + bp + extra) / dt / 1e9
    check_peak("autograd step", gbs)
    gbs_csr = (sum(plain_bytes(ddc.info, 1, csr_equivalent=True)) + extra) / dt / 1e9
    log(f"F = {float(F):.6g}; forward+backward {dt * 1e3:.3f} ms ({gbs:.0f} GB/s)")
    print(json.dumps({
        "metric": "effective HBM GB/s of one autograd evaluation of F(D B y) and dF/dy",
        "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(dt * 1e3, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": storage, "data": "synthetic",
        "config": {"workload": plan.name, "n_vox": plan.n_vox, "n_beamlets": plan.n_bl, "nnz": int(ddc.info.nnz),
                   "apertures": 64, "storage": storage, "pct_hbm_peak": round(100.0 * gbs / HBM_PEAK_GBS, 2),
                   "csr_equivalent_gbs": round(gbs_csr, 2),
                   "generate_s": round(t_gen, 1), "build_upload_s": round(t_build, 1)},
    }), flush=True)


def bench_shard(args):
    """One GPU's share of a split by voxel rows: the z-slab of the two-arc
    workload that a GPU of --shards would hold (slabs cut for equal entry
    counts, or equal thickness with --slabs equal; the heaviest slab is timed),
    with its dose (objective epilogue) and its partial price timed at that real
    shape.  The exchange the split needs (the price summed over the GPUs, n_bl
    floats) is not run here."""
    import numpy as np
    import torch
    from paper_1503_01721_amd import dvmat, synth
    workload = args.workload if args.workload != "cp180_bl40x40_vox128" else "cp360_bl60x60_vox160"
    storage = args.storage if "--storage" in sys.argv else "f16"
    plan = synth.PLANS[workload]
    N, G = plan.n_grid, args.shards
    if G < 1 or G > N:
        raise SystemExit(f"--shards must be between 1 and the {N} voxel slices")
    counts = synth.slice_counts(plan)
    if args.slabs == "balanced":
        slabs = synth.balanced_slabs(plan, G, counts)
    else:
        slabs = [(k * N // G, (k + 1) * N // G) for k in range(G)]
    share = [int(counts[a:b].sum()) for a, b in slabs]
    s = int(np.argmax(share))                                # the heaviest slab sets the pace
    z0, z1 = slabs[s]
    log(f"{args.slabs} slabs {slabs}; entries per slab {share}")
    t = time.perf_counter()
    d = synth.generate_ddc(plan, z_slab=(z0, z1))
    d["row"] -= z0 * N * N                                   # slab-local voxel rows
    sid, table = synth.structures(plan)
    sid = sid[z0 * N * N:z1 * N * N]
    n_vox = (z1 - z0) * N * N
    t_gen = time.perf_counter() - t
    log(f"generated slab {s} of {G} (slices {z0}..{z1 - 1}) of {plan.name}: nnz={len(d['val'])} in {t_gen:.1f} s")
    t = time.perf_counter()
    layout = grid_layout(args, {"dose_grid": (N, N, z1 - z0), "price_grid": plan.grids["price_grid"]})
    # a thin slab leaves each beamlet row a few hundred entries: the sliced
    # layout (the default with grids) runs such short rows in lock step; in
    # CSR two rows per block row halve the reductions
    if args.layout == "csr":
        layout["price_block_rows"] = 2
    ddc = dvmat.DDC(d["row"], d["col"], d["val"], n_vox, plan.n_bl, storage=storage, **layout)
    del d
    obj = dvmat.Objective(sid, table)
    t_build = time.perf_counter() - t
    if not args.no_autotune:
        ddc.autotune(reps=3)
    x, g = synth.bench_vectors(plan.n_bl, n_vox, 1004)
    x = torch.from_numpy(x).cuda()
    g0 = torch.from_numpy(g).cuda()
    z = torch.empty(n_vox, device="cuda")
    gz = torch.empty(n_vox, device="cuda")
    F = torch.empty(1, device="cuda")
    p = torch.empty(plan.n_bl, device="cuda")
    for _ in range(max(args.warmup, 1)):
        ddc.dose_(x, z, obj, gz, F)
        ddc.price_(g0, p)
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    ev[0].record()
    for _ in range(args.steps):
        ddc.dose_(x, z, obj, gz, F)
    ev[1].record()
    for _ in range(args.steps):
        ddc.price_(g0, p)
    ev[2].record()
    torch.cuda.synchronize()
    td = ev[0].elapsed_time(ev[1]) / args.steps
    tp = ev[1].elapsed_time(ev[2]) / args.steps
    b = algorithmic_bytes(ddc.info)
    gbs = (b["dose"] + b["price"]) / ((td + tp) * 1e-3) / 1e9
    check_peak("slab dose + price", gbs)
    bc = algorithmic_bytes(ddc.info, csr_equivalent=True)
    gbs_csr = (bc["dose"] + bc["price"]) / ((td + tp) * 1e-3) / 1e9
    allreduce_us = 2.0 * (G - 1) / G * 4 * plan.n_bl / 153e9 * 1e6
    log(f"slab dose {td:.3f} ms, partial price {tp:.3f} ms ({gbs:.0f} GB/s); "
        f"ring all-reduce of the price over {G} GPUs at 153 GB/s per link: ~{allreduce_us:.0f} us (estimate)")
    print(json.dumps({
        "metric": "effective HBM GB/s of one GPU's share (voxel-row split) of D.x + D^T.g",
        "value": round(gbs, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(td + tp, 4), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": storage, "data": "synthetic",
        "config": {"workload": f"{plan.name}, voxel slab {s} of {G} (slices {z0}..{z1 - 1}, {args.slabs} slabs)",
                   "n_vox": n_vox, "nnz_total": int(counts.sum()),
                   "n_beamlets": plan.n_bl, "nnz": int(ddc.info.nnz), "storage": storage,
                   "dose_ms": round(td, 4), "price_ms": round(tp, 4), "csr_equivalent_gbs": round(gbs_csr, 2),
                   "pct_hbm_peak": round(100.0 * gbs / HBM_PEAK_GBS, 2),
                   "price_allreduce_us_estimate": round(allreduce_us, 1),
                   "generate_s": round(t_gen, 1), "build_upload_s": round(t_build, 1)},
    }), flush=True)


def plan_metrics(z, sid_dev, ptv_ids, table):
    """Dose summary of a plan (reporting only): per PTV the mean dose and the
    fraction of its voxels above 110 % of its prescription (Table 1's
    criterion); per OAR the maximum dose."""
    import torch
    from paper_1503_01721_amd import synth
    out = {}
    for k in ptv_ids:
        m = sid_dev == k
        zk = z[m]
        rx = float(table[k][0])
        out[f"ptv{k - synth.S_PTV0}"] = {"mean": round(float(zk.mean()), 3),
                                         "v110_pct": round(100.0 * float((zk > 1.1 * rx).float().mean()), 2)}
    for name, k in (("oar_a", synth.S_OAR_A), ("oar_b", synth.S_OAR_B)):
        m = sid_dev == k
        out[name] = {"max": round(float(z[m].max()), 3) if bool(m.any()) else None,
                     "threshold": float(table[k][0])}
    return out


def bench_truncation(args):
    """The truncation study of Sec. 2.4 (S1) and Sec. 3: column generation on
    a matrix truncated by a cone of radius gamma about each beamlet axis (here
    a cylinder: the beams are parallel), then the plan's actual dose on the
    complete matrix.  The complete matrix's own cut-off (1e-3 of the kernel
    maximum) reaches 11.15 mm from the axis; the paper's complete-to-truncated
    cone ratio (6 cm to 2.5 cm) corresponds to about 4.5 mm here."""
    import torch
    from paper_1503_01721_amd import dvmat, synth
    from paper_1503_01721_amd.colgen import ColumnGeneration
    # the dose study runs on the plain-method workload by default: with the
    # generator's attenuation (0.05 per mm) a 30-iteration plan at full scale
    # leaves the central target at a few Gy, where a dose shift means nothing;
    # --workload cp180_bl40x40_vox128 gives the per-iteration times at full scale
    workload = args.workload if "--workload" in sys.argv else "cp20_bl20x20_vox32"
    plan = synth.PLANS[workload]
    cones = [None] + [float(c) for c in args.cones.split(",") if c]
    sid, table = synth.structures(plan)
    sid_dev = torch.from_numpy(sid).cuda()
    ptv_ids = [k for k in range(synth.S_PTV0, len(table))]
    obj = dvmat.Objective(sid, table)
    layout = grid_layout(args, plan.grids)
    iters = args.warmup + args.steps
    rows, full_ddc, ref_nnz = [], None, None
    for cone in cones:
        t = time.perf_counter()
        d = synth.generate_ddc(plan, cone_mm=cone)
        ddc = dvmat.DDC(d["row"], d["col"], d["val"], plan.n_vox, plan.n_bl, storage=args.storage, **layout)
        del d
        t_build = time.perf_counter() - t
        if cone is None:
            full_ddc, ref_nnz = ddc, ddc.info.nnz
        if not args.no_autotune:
            ddc.autotune(reps=3)
        cg = ColumnGeneration(ddc, obj, plan.n_cp, plan.n_rows, plan.n_cols, max_apertures=iters,
                              bb_steps=args.bb_steps)
        cg.start()
        for _ in range(args.warmup):
            cg.iteration()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            if cg.iteration() is None:
                break
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / max(1, args.steps) * 1e3
        z_opt = cg.z.clone()
        z_act = full_ddc.dose(cg.x)
        F_opt = float(obj(z_opt, with_grad=False)[0][0])
        F_act = float(obj(z_act, with_grad=False)[0][0])
        opt, act = plan_metrics(z_opt, sid_dev, ptv_ids, table), plan_metrics(z_act, sid_dev, ptv_ids, table)
        shift = 100.0 * (act["ptv0"]["mean"] / opt["ptv0"]["mean"] - 1.0)
        row = {"cone_mm": cone, "nnz": int(ddc.info.nnz), "nnz_frac": round(ddc.info.nnz / ref_nnz, 4),
               "ms_per_iteration": round(ms, 3), "iterations": len(cg.records), "F_optimised": F_opt,
               "F_actual": F_act, "ptv_mean_shift_pct": round(shift, 2), "optimised": opt, "actual": act,
               "build_s": round(t_build, 1)}
        rows.append(row)
        log(f"cone {cone} mm: nnz {ddc.info.nnz} ({row['nnz_frac']:.3f}), {ms:.2f} ms/iteration, "
            f"PTV mean {opt['ptv0']['mean']:.2f} optimised -> {act['ptv0']['mean']:.2f} actual ({shift:+.1f} %), "
            f"V110 {opt['ptv0']['v110_pct']} -> {act['ptv0']['v110_pct']} %, F {F_opt:.6g} -> {F_act:.6g}")
        del cg
        if cone is not None:
            del ddc
        torch.cuda.synchronize()
    pick = min((r for r in rows if r["cone_mm"] is not None), key=lambda r: abs(r["cone_mm"] - 4.5), default=rows[0])
    print(json.dumps({
        "metric": "truncation study: actual minus optimised mean PTV dose (%) of a plan optimised on a "
                  "cone-truncated DDC matrix",
        "value": pick["ptv_mean_shift_pct"], "unit": "%", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": pick["ms_per_iteration"], "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": args.storage, "data": "synthetic",
        "config": {"workload": plan.name, "cone_mm_reported": pick["cone_mm"], "layout": args.layout,
                   "bb_steps_per_iteration": args.bb_steps, "rows": rows},
    }), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed column-generation iterations")
    ap.add_argument("--warmup", type=int, default=2, help="untimed iterations before the timed ones")
    ap.add_argument("--workload", default="cp180_bl40x40_vox128")
    ap.add_argument("--storage", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--bb-steps", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default launch shape")
    ap.add_argument("--dose-kernel", default=None, metavar="KIND:WG",
                    help="fix the dose launch (e.g. row:1024) instead of autotuning it")
    ap.add_argument("--price-kernel", default=None, metavar="KIND:WG",
                    help="fix the price launch (e.g. row:8192) instead of autotuning it")
    ap.add_argument("--mode", default="colgen", choices=["colgen", "batched", "autograd", "shard", "truncation"],
                    help="colgen: column-generation iterations (default); batched: many plans x 8 "
                         "right-hand sides in one launch vs one plan at a time; autograd: F(D B y) "
                         "forward + backward on the two-arc workload; shard: one GPU's voxel slab of "
                         "the two-arc workload (--shards); truncation: plans optimised on cone-truncated "
                         "matrices (--cones) re-evaluated on the complete one")
    ap.add_argument("--cones", default="9,7.5,6,4.5", help="cone radii (mm) of --mode truncation")
    ap.add_argument("--shards", type=int, default=8, help="GPUs of the voxel-row split in --mode shard")
    ap.add_argument("--slabs", default="balanced", choices=["balanced", "equal"],
                    help="voxel slabs of --mode shard: equal entry counts (default) or equal thickness")
    ap.add_argument("--plans", type=int, default=48, help="plans in --mode batched")
    ap.add_argument("--batch-price-layout", default="csr", choices=["csr", "panel", "sliced"],
                    help="layout of the price orientation in --mode batched")
    ap.add_argument("--batch-dose-layout", default="sliced", choices=["panel", "sliced"],
                    help="layout of the dose orientation in --mode batched")
    ap.add_argument("--batch-dose-b", type=int, default=1, help="rows per block row of the dose in --mode batched")
    ap.add_argument("--batch-price-b", type=int, default=0,
                    help="rows per block row of the price in --mode batched (0: the library's default)")
    ap.add_argument("--panel-cols", type=int, default=3584,
                    help="column budget of the dose panels in --mode batched (3584: 4 right-hand sides per launch)")
    ap.add_argument("--form", default="D", choices=["D", "DA"],
                    help="master problem over the whole matrix (D, default: every BB iteration runs "
                         "a dose and a price product) or over the aperture dose vectors (DA)")
    ap.add_argument("--layout", default="grid", choices=["grid", "sliced", "panel", "csr"],
                    help="device layout of both orientations: grid (default: the tuner's cached choice of "
                         "panel layouts, else the library's default, sliced panels), sliced or panel forced "
                         "(vector slices staged in LDS), or CSR (gathers from global memory)")
    ap.add_argument("--dose-lanes", type=int, default=0, choices=[0, 4, 8, 16],
                    help="sliced layout: lanes per dose row (0: the library's default)")
    ap.add_argument("--price-lanes", type=int, default=0, choices=[0, 4, 8, 16],
                    help="sliced layout: lanes per price row (0: the library's default)")
    ap.add_argument("--tune", action="store_true",
                    help="time the candidate layouts first and cache the fastest (DVMAT_TUNE_CACHE)")
    ap.add_argument("--no-tuned-layout", action="store_true", help="ignore the tuner cache: library defaults")
    ap.add_argument("--no-graph", action="store_true",
                    help="DA form: launch the master problem's kernels one by one instead of replaying a captured graph")
    ap.add_argument("--copy-calibration", action="store_true", help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the whole DDC matrix fits one MI355X's HBM); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    if args.copy_calibration:
        copy_calibration()
        return

    from paper_1503_01721_amd import dvmat, synth, tuner
    from paper_1503_01721_amd.colgen import ColumnGeneration

    if args.mode == "batched":
        return bench_batched(args)
    if args.mode == "autograd":
        return bench_autograd(args)
    if args.mode == "shard":
        return bench_shard(args)
    if args.mode == "truncation":
        return bench_truncation(args)

    plan = synth.PLANS[args.workload]
    if args.warmup + args.steps > plan.n_cp:
        raise SystemExit("more iterations than control points")
    log(f"generating {plan.name}: {plan.n_vox} voxels x {plan.n_bl} beamlets")
    t = time.perf_counter()
    d = synth.generate_ddc(plan)
    sid, table = synth.structures(plan)
    t_gen = time.perf_counter() - t
    log(f"generated nnz={len(d['val'])} in {t_gen:.1f} s")

    obj = dvmat.Objective(sid, table)
    layout = grid_layout(args, plan.grids)
    layout_source = "csr" if args.layout == "csr" else "defaults" if args.layout == "grid" else "forced"
    if args.layout == "grid":
        # the layout knobs (tiles, block rows, panel budget, part size) come from
        # the tuner: its cache, or a tuning run now with --tune
        sig = tuner.signature(plan.n_vox, plan.n_bl, len(d["val"]), args.storage, plan.grids, 1)
        tuned = None
        if args.tune:
            tuned = tuner.tune(d["row"], d["col"], d["val"], plan.n_vox, plan.n_bl, args.storage, plan.grids, obj,
                               log=log)
        elif not args.no_tuned_layout:
            tuned = tuner.layout_for(sig)
        if tuned:
            layout.update(tuned)
            layout_source = "tuner"
            log(f"layout from the tuner ({tuner.cache_path()}): {tuned}")
        else:
            log(f"no tuned layout for {sig}: library defaults")
    t = time.perf_counter()
    ddc = dvmat.DDC(d["row"], d["col"], d["val"], plan.n_vox, plan.n_bl, storage=args.storage, **layout)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - t
    info = ddc.info
    log(f"built CSR(D) + CSR(D^T) and uploaded {info.workspace_bytes / 2**30:.2f} GiB in {t_build:.1f} s")
    fixed = {"dose": args.dose_kernel, "price": args.price_kernel}
    if not args.no_autotune and not any(fixed.values()):
        t = time.perf_counter()
        info = ddc.autotune(reps=5, obj=obj)
        log(f"autotuned in {time.perf_counter() - t:.1f} s: dose kernel {('row', 'stream', 'pipe', 'panel')[info.dose_kernel]} "
            f"x {info.dose_workgroups} wg ({info.dose_tuned_ms:.3f} ms), price kernel "
            f"{('row', 'stream', 'pipe', 'panel')[info.price_kernel]} x {info.price_workgroups} wg ({info.price_tuned_ms:.3f} ms)")
    for orient, spec in fixed.items():
        if spec:
            kind, wg = spec.split(":")
            ddc.set_kernel(orient, kind, int(wg))
            info = ddc.refresh_info()
            log(f"{orient} launch fixed at {kind} x {wg} workgroups")

    # the DA form's master problem is many small launches: captured once in a
    # HIP graph and replayed per iteration; the D form's is 101 launches over
    # the whole matrix, timed one by one with events
    graph = args.form == "DA" and not args.no_graph
    cg = ColumnGeneration(ddc, obj, plan.n_cp, plan.n_rows, plan.n_cols,
                          max_apertures=args.warmup + args.steps, bb_steps=args.bb_steps, form=args.form,
                          graph=graph)
    cg.start()
    for i in range(args.warmup):
        rec = cg.iteration()
        log(f"warmup iteration {i}: {rec}")
    torch.cuda.synchronize()

    cg.events = None if graph else []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        # one read-back per iteration: this iteration's F and flags come with the next
        rec = cg.iteration(sync=False)
        if rec is None:
            raise SystemExit("column generation stopped inside the timed region")
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    cg.finish()
    wall = t1 - t0
    log(f"timed {args.steps} iterations in {wall:.3f} s; last {cg.records[-1]}")

    ab = algorithmic_bytes(info)
    abc = algorithmic_bytes(info, csr_equivalent=True)

    def iteration_bytes(b):
        if args.form == "D":
            return args.bb_steps * (b["dose"] + b["price"]) + b["curv"]
        # one price product and one dose product (the new aperture's column) per
        # iteration; the BB iterations read the DA columns, not the matrix
        return b["price"] + b["dose"]
    per_iter = iteration_bytes(ab)
    value = args.steps * per_iter / wall / 1e9
    value_csr = args.steps * iteration_bytes(abc) / wall / 1e9
    check_peak("whole job", value)
    if not cg.events:
        cg.events = []
    if not cg.events:
        # DA form: time one dose and one price product beside the iterations
        x_t = torch.rand(plan.n_bl, device="cuda")
        z_t = torch.empty(plan.n_vox, device="cuda")
        g_t = torch.empty(plan.n_vox, device="cuda")
        F_t = torch.empty(1, device="cuda")
        p_t = torch.empty(plan.n_bl, device="cuda")
        for _ in range(5):
            e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
            e[0].record()
            ddc.dose_(x_t, z_t, obj, g_t, F_t)
            e[1].record()
            ddc.price_(g_t, p_t)
            e[2].record()
            cg.events.append(e)
        torch.cuda.synchronize()
    dose_ms = [e[0].elapsed_time(e[1]) for e in cg.events]
    price_ms = [e[1].elapsed_time(e[2]) for e in cg.events]
    mean_dose = sum(dose_ms) / len(dose_ms)
    mean_price = sum(price_ms) / len(price_ms)
    dom = "price" if mean_price >= mean_dose else "dose"
    dom_ms = mean_price if dom == "price" else mean_dose
    achieved = ab[dom] / (dom_ms * 1e-3) / 1e9
    check_peak("dose kernel", ab["dose"] / mean_dose / 1e6)
    check_peak("price kernel", ab["price"] / mean_price / 1e6)
    dom_layout = info.price_layout if dom == "price" else info.dose_layout
    kfn = KERNEL_NAMES[dom_layout]
    kname = (f"{kfn} (price, D^T in the {LAYOUT_NAMES[dom_layout]} layout)" if dom == "price"
             else f"{kfn} (dose, D in the {LAYOUT_NAMES[dom_layout]} layout, objective epilogue)")
    traffic = read_traffic(dom, plan.name, args.storage, LAYOUT_NAMES[dom_layout])
    log(f"mean dose call {mean_dose:.3f} ms ({ab['dose'] / mean_dose / 1e6:.0f} GB/s), "
        f"mean price call {mean_price:.3f} ms ({ab['price'] / mean_price / 1e6:.0f} GB/s)")

    out = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.storage,
        "data": "synthetic",
        "config": {
            "workload": plan.name,
            "n_vox": plan.n_vox, "n_beamlets": plan.n_bl, "nnz": int(info.nnz),
            "storage": args.storage, "accumulate": "f32", "bb_steps_per_iteration": args.bb_steps,
            "master_problem_form": args.form, "master_problem_graph": graph,
            "products_per_iteration": 2 * args.bb_steps + 1 if args.form == "D" else 2,
            "algorithmic_bytes_per_iteration": per_iter,
            "algorithmic_bytes_per_launch": {"dose": ab["dose"], "price": ab["price"], "curvature": ab["curv"]},
            "index_bytes_per_nnz": {"dose": index_bytes(info, "dose"), "price": index_bytes(info, "price")},
            "pct_hbm_peak": round(100.0 * value / HBM_PEAK_GBS, 2),
            "csr_equivalent_gbs": round(value_csr, 2),
            "dose_gbs": round(ab["dose"] / mean_dose / 1e6, 1), "price_gbs": round(ab["price"] / mean_price / 1e6, 1),
            "mean_dose_call_ms": round(mean_dose, 4), "mean_price_call_ms": round(mean_price, 4),
            "generate_s": round(t_gen, 2), "build_upload_s": round(t_build, 2),
            "layout": {"dose": LAYOUT_NAMES[info.dose_layout], "price": LAYOUT_NAMES[info.price_layout]},
            "layout_source": layout_source,
            "layout_options": {k: v for k, v in layout.items() if k not in ("dose_grid", "price_grid")},
            "dose_panels": int(info.dose_panels), "price_panels": int(info.price_panels),
            "dose_launch": {"kernel": ("row", "stream", "pipe", "panel")[info.dose_kernel], "workgroups": info.dose_workgroups},
            "price_launch": {"kernel": ("row", "stream", "pipe", "panel")[info.price_kernel], "workgroups": info.price_workgroups},
        },
        "roofline": {
            "bound": "hbm", "kernel": kname,
            "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": ab[dom], "mean_launch_ms": round(dom_ms, 4),
            "csr_equivalent_gbs": round(abc[dom] / (dom_ms * 1e-3) / 1e9, 1),
        },
    }
    if not args.no_cpu_baseline:
        log("timing the FP64 oracle on dose and price product pairs (CPU baseline)")
        bplain = ab["dose"] - info.n_vox * (1 + 4)
        out["cpu_baseline"] = cpu_baseline(d, plan, bplain, ab["price"])
        log(f"cpu baseline {out['cpu_baseline']['value']} GB/s in {out['cpu_baseline']['seconds']} s")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
