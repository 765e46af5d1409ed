#!/usr/bin/env python3
"""PLSS benchmark on one MI355X.

Workload (default): the large consistent system, 2,000,000 x 500,000, row
lengths Zipf(1.5) clipped to [2, 2000] (nnz ~1.37e8), N(0,1) values,
x* ~ N(0,1), b = A x*, residual sketch (Algorithm 1), FP64, relative
tolerance 1e-8, maxit 1000.  One step = one full solve; A, b and x stay
resident in HBM (torch device tensors) during the timed region.

Reported: PLSS iterations/s (value), solves/s, algorithmic HBM GB/s of the
iteration, the roofline of the dominant kernel (per-kernel HIP events on
the library's stream during the timed region, around the phases of one
iteration in eight so that the events barely slow the others), the oracle
timed on the host
on a bounded sample, and two more arms of the same system timed separately
after the main region: float32 storage + float64 refinement, and PLSS W
(W = diag(1/||A_{:,j}||), Section 4.1).

    python bench.py [--gpus 1] [--steps 10] [--warmup 2]
    python bench.py --config small|underdet|batch|multi|serve   (other workloads)
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("PLSS iters/s & HBM GB/s (SpMV+SpMVᵀ); solves/s, p50/p99 at rel. res 1e-8")
HBM_PEAK_GBS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def bytes_model(m, n, nnz, f32=False):
    """Algorithmic bytes per iteration and per kernel (int32 pointers and
    indices; float64 vectors, or float32 vectors for float32 storage):
      product with A  : v*nnz + 4*nnz + 4m (ptr) + 2w*m (r read+write) + w*n (p)
      product with Aᵀ : v*nnz + 4*nnz + 4n (ptr) + w*n (y write) + w*m (r)
      update          : 5w*n (p read+write, y read, x read+write; x in f64)"""
    v = 4 if f32 else 8
    w = 4 if f32 else 8
    spmv = (v + 4) * nnz + 4 * m + 2 * w * m + w * n
    spmvt = (v + 4) * nnz + 4 * n + w * n + w * m
    upd = 3 * w * n + 16 * n
    return {"spmv": spmv, "spmvt": spmvt, "update": upd, "iter": spmv + spmvt + upd}


def recorded_traffic(kernel_index, layout):
    """Calibrated HBM bytes per launch of the dominant kernel from the
    committed rocprofv3 counter passes, or None when the kernel source (or
    the layout) differs from the one the counters were taken with."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "large_fp64_traffic.txt")
    try:
        kv = dict(l.strip().split("=", 1) for l in open(path) if "=" in l and not l.startswith("#"))
        h = hashlib.sha1()
        for name in kv["sources"].split(","):
            h.update(open(os.path.join(ROOT, "paper_2207_07615_amd", "csrc", name), "rb").read())
        if kv.get("sources_sha1_12") != h.hexdigest()[:12] or kv.get("layout") != layout:
            return None
        sfx = "" if kernel_index == 0 else "_t"
        return (float(kv["fetch_kib" + sfx]) * float(kv["fetch_scale"]) +
                float(kv["write_kib" + sfx]) * float(kv["write_scale"])) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(sysm, iters=60, threads=1):
    """The oracle (Algorithm 1 in float64, SciPy sparse products) on the
    first `iters` iterations of the same system, with the host's thread
    pools (BLAS / OpenMP) limited to `threads`.  SciPy's sparse products run
    on one thread whatever the limit; only NumPy's dense dots use the pool."""
    from threadpoolctl import threadpool_limits, threadpool_info
    from oracle import plss as O
    with threadpool_limits(threads):
        pool = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
        t0 = time.perf_counter()
        res = O.plss_residual(sysm.A, sysm.b, tol=1e-300, maxit=iters)
        dt = time.perf_counter() - t0
    return {"value": res.iters / dt, "unit": "iters/s", "cores": pool, "kind": "oracle",
            "sample": f"first {res.iters} iterations of the same float64 solve "
                      f"({dt:.1f} s, SciPy CSR products on one thread, NumPy dots on "
                      f"{pool} thread{'s' if pool > 1 else ''})"}


def _gen_batch(i):
    import plss_inputs as gen
    import numpy as np
    s = gen.batch_systems(1, first=i)[0]
    A32 = s.A.astype(np.float32)
    return A32, gen.rhs(A32, s.xstar), s.xstar


def _gen_stream(i):
    import plss_inputs as gen
    import numpy as np
    s = gen.stream_systems(1, first=i)[0]
    A32 = s.A.astype(np.float32)
    return s, A32, gen.rhs(A32, s.xstar)


def _pool_map(fn, items):
    import concurrent.futures as cf
    workers = min(16, os.cpu_count() or 4)
    with cf.ProcessPoolExecutor(max_workers=workers) as ex:
        return list(ex.map(fn, items, chunksize=1))


def base_line(metric, value, unit, steps, warmup, wall, dtype, config, **extra):
    out = {"metric": metric, "value": value, "unit": unit, "n_gpus": 1, "steps": steps,
           "warmup": warmup, "ms_per_step": 1e3 * wall / max(1, steps), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": dtype,
           "data": "synthetic (seeded; stands in for the paper's datasets)", "config": config}
    out.update(extra)
    return out


def kernel_roofline(kms, kn, bm, kind="spmv"):
    avg = [kms[q] / max(1, kn[q]) for q in range(4)]
    dom = 0 if avg[0] >= avg[1] else 1
    dom_bytes = bm["spmv"] if dom == 0 else bm["spmvt"]
    ach = dom_bytes / (avg[dom] * 1e-3) / 1e9 if avg[dom] > 0 else 0.0
    return avg, {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": ach / HBM_PEAK_GBS, "traffic": None,
                 "kernel": ("product with A" if dom == 0 else "product with Aᵀ") + f" ({kind})",
                 "algorithmic_bytes_per_launch": dom_bytes}


def run_small(args):
    """2000 x 1000, 8 nnz per row, FP64, tol 1e-8.  The automatic engine
    solves this system in one workgroup (vectors in LDS, matrix in L2), so
    one kernel runs the whole solve: its device time per solve gives the
    roofline line (cache-resident data: the fraction is against HBM peak
    but the bytes come from L2).  The one-launch-per-phase engine is timed
    beside it."""
    import numpy as np
    import paper_2207_07615_amd as plss
    import plss_inputs as gen
    from oracle import plss as O
    import torch
    sysm = gen.small()
    A = sysm.A
    h = plss.Handle(0)
    M = plss.Matrix(h, A.row_ptr, A.col_idx, A.vals, shape=(A.m, A.n))
    b_d = torch.from_numpy(sysm.b).to(torch.device("cuda:0"))  # b and x stay in HBM
    torch.cuda.synchronize()
    kw = dict(tol=1e-8, maxit=1000)
    for _ in range(args.warmup):
        plss.solve(h, M, b_d, **kw)
    lat, its, dev = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        x, info, _ = plss.solve(h, M, b_d, **kw)
        lat.append(time.perf_counter() - ts)
        its.append(info["iters"])
        dev.append(info["ms"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    x = x.cpu().numpy()
    # the per-phase engine on the same system, for comparison
    plss.solve(h, M, b_d, engine="multi", **kw)
    tm = time.perf_counter()
    itm = 0
    for _ in range(args.steps):
        _, im, _ = plss.solve(h, M, b_d, engine="multi", **kw)
        itm += im["iters"]
    torch.cuda.synchronize()
    wm = time.perf_counter() - tm
    bm = bytes_model(A.m, A.n, A.nnz)
    dev_ms = sum(dev) / len(dev)
    iters = sum(its) / len(its)
    ach = bm["iter"] * iters / (dev_ms * 1e-3) / 1e9
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBS,
            "traffic": None, "kernel": "k_small<double,double> (whole solve in one workgroup)",
            "algorithmic_bytes_per_launch": bm["iter"] * iters}
    # oracle: repeated full solves for about 5 s of one host thread
    t1 = time.perf_counter()
    nref = 0
    while True:
        ref = O.plss_residual(A, sysm.b, tol=1e-8, maxit=1000)
        nref += 1
        if time.perf_counter() - t1 > 5.0:
            break
    tc = time.perf_counter() - t1
    lat = sorted(1e3 * v for v in lat)
    return base_line(METRIC, sum(its) / wall, "iters/s", args.steps, args.warmup, wall, "f64",
                     {"workload": "small: 2000 x 1000 CSR, 8 nnz/row, N(0,1), residual sketch, FP64, tol 1e-8",
                      "m": A.m, "n": A.n, "nnz": A.nnz, "engine": "single workgroup (automatic)"},
                     solves_per_s=args.steps / wall, iters_per_solve=iters,
                     p50_ms=lat[len(lat) // 2], p99_ms=lat[-1], relres_true=info["relres_true"],
                     device_ms_per_solve=dev_ms, device_us_per_iter=1e3 * dev_ms / iters,
                     per_phase_engine_iters_per_s=itm / wm, roofline=roof,
                     rel_err_vs_oracle=float(np.linalg.norm(x - ref.x) / np.linalg.norm(ref.x)),
                     cpu_baseline={"value": nref * ref.iters / tc, "unit": "iters/s", "cores": 1, "kind": "oracle",
                                   "sample": f"{nref} full solves of {ref.iters} iterations ({tc:.1f} s)"})


def column_bytes(m, n, nnz, kh, residual):
    """Algorithmic bytes of one one-column sketch step with kh stored
    updates (float64, int32 indices): a residual column adds y = Aᵀ r
    (12 nnz + 4n + 8n + 8m) and (AP)ᵀ r (8 m kh + 8m); every column reads P
    for p = gamma (y - P c) (8 n kh + 8n, writes p and updates x: 24n) and
    runs A p into AP and r (12 nnz + 4m + 8n + 8m + 16m)."""
    b = 8 * n * kh + 8 * n + 24 * n + 12 * nnz + 4 * m + 8 * n + 24 * m
    if residual:
        b += 12 * nnz + 12 * n + 8 * m + 8 * m * kh + 8 * m
    return b


def block_bytes(m, n, nnz, K, w, residual):
    """Algorithmic bytes of one block step with K stored history columns and
    w columns in the block: [y = Aᵀ r and (A Z)ᵀ r: 12 nnz + 12n + 8m +
    8 m K + 8m]; Z_new = Y_new - Z C reads Z and y, writes Z_new, updates x
    (8 n K + 8n + 8 n w + 16n); A Z_new into the history and r (12 nnz + 4m +
    8 n w + 8 m w + 16m)."""
    b = 8 * n * K + 8 * n + 8 * n * w + 16 * n + 12 * nnz + 4 * m + 8 * n * w + 8 * m * w + 16 * m
    if residual:
        b += 12 * nnz + 12 * n + 8 * m + 8 * m * K + 8 * m
    return b


def run_underdet(args):
    """200,000 x 1,000,000, 30 nnz per row, U(-1,1), mixed sketch, FP64; and
    the same system with mixed blocks of 15 rows (16 columns per step)."""
    import numpy as np
    import paper_2207_07615_amd as plss
    import plss_inputs as gen
    from oracle import plss as O
    import torch
    sysm = gen.underdet()
    A = sysm.A
    h = plss.Handle(0)
    M = plss.Matrix(h, A.row_ptr, A.col_idx, A.vals, shape=(A.m, A.n))
    # b, the row order and x stay in HBM (device tensors) in the timed region
    gpu = torch.device("cuda:0")
    b_d = torch.from_numpy(sysm.b).to(gpu)
    perm_d = torch.from_numpy(sysm.perm).to(gpu)
    torch.cuda.synchronize()
    kw = dict(sketch="mixed", tol=1e-8, maxit=2000, row_perm=perm_d, hist_cap=128)
    for _ in range(args.warmup):
        plss.solve(h, M, b_d, **kw)
    its, dev, cols = [], [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        x, info, _ = plss.solve(h, M, b_d, **kw)
        its.append(info["iters"])
        dev.append(info["ms"])
        cols.append(info["outer_iters"])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the same solves handed host buffers (b and the row order copied in, x
    # copied out on every call): the rate with the PCIe transfers
    kwh = dict(kw, row_perm=sysm.perm)
    th = time.perf_counter()
    for _ in range(3):
        plss.solve(h, M, sysm.b, **kwh)
    host_ms = 1e3 * (time.perf_counter() - th) / 3
    # bytes of the columns of one solve: columns alternate residual / identity,
    # the history holds the updates so far (no skip, no clear at this size)
    nupd = its[-1]
    col_b = sum(column_bytes(A.m, A.n, A.nnz, t // 2, t % 2 == 0) for t in range(cols[-1]))
    # mixed blocks of 15 identity rows plus r (one MFMA tile of 16 columns)
    kwb = dict(sketch="block_mixed", block=15, tol=1e-8, maxit=2000, row_perm=perm_d, hist_cap=256)
    for _ in range(args.warmup):
        plss.solve(h, M, b_d, **kwb)
    itb, devb = [], []
    t1 = time.perf_counter()
    for _ in range(args.steps):
        xb, ib, _ = plss.solve(h, M, b_d, **kwb)
        itb.append(ib["iters"])
        devb.append(ib["ms"])
    torch.cuda.synchronize()
    wallb = time.perf_counter() - t1
    blk_b = sum(block_bytes(A.m, A.n, A.nnz, 16 * (t % 16), 16, True) for t in range(itb[-1]))
    t2 = time.perf_counter()
    ref = O.plss_columns(A, sysm.b, "mixed", perm=sysm.perm, tol=1e-300, maxit=8, hist_cap=128)
    tc = time.perf_counter() - t2
    x8, i8, _ = plss.solve(h, M, sysm.b, sketch="mixed", tol=1e-300, maxit=8, row_perm=sysm.perm, hist_cap=128)
    x8 = np.asarray(x8)
    return base_line(METRIC, sum(its) / wall, "updates/s", args.steps, args.warmup, wall, "f64",
                     {"workload": "underdet: 200,000 x 1,000,000 CSR, 30 nnz/row, U(-1,1), mixed sketch "
                                  "(residual + identity columns), FP64, tol 1e-8",
                      "m": A.m, "n": A.n, "nnz": A.nnz, "hist_cap": 128},
                     solves_per_s=args.steps / wall, updates_per_solve=sum(its) / len(its),
                     columns_per_solve=sum(cols) / len(cols),
                     device_ms_per_solve=sum(dev) / len(dev),
                     host_buffers_ms_per_solve=host_ms,
                     relres_true=info["relres_true"], status=info["status_name"],
                     roofline=aggregate_roofline(col_b * args.steps, wall, "whole solves (all column steps)"),
                     rel_err_vs_oracle_8_updates=float(np.linalg.norm(x8 - ref.x) / np.linalg.norm(ref.x)),
                     mixed_blocks_15={"solves_per_s": args.steps / wallb, "ms_per_solve": 1e3 * wallb / args.steps,
                                      "block_steps_per_solve": sum(itb) / len(itb),
                                      "device_ms_per_solve": sum(devb) / len(devb),
                                      "relres_true": ib["relres_true"], "status": ib["status_name"],
                                      "hist_cap": 256,
                                      "roofline": aggregate_roofline(blk_b * args.steps, wallb,
                                                                     "whole solves (all block steps)"),
                                      "solves_per_s_vs_one_column": (args.steps / wallb) / (args.steps / wall)},
                     cpu_baseline={"value": ref.iters / tc, "unit": "updates/s", "cores": 1, "kind": "oracle",
                                   "sample": f"first {ref.iters} column steps ({tc:.1f} s)"})


def host_relres(A, b, x):
    """||b - A x|| / ||b|| on the host (SciPy, float64): the check every
    counted solve must pass."""
    import numpy as np
    nb = float(np.linalg.norm(b))
    r = float(np.linalg.norm(b - A.scipy() @ x))
    return r / nb if nb > 0 else r


def aggregate_roofline(byte_total, wall, what):
    """Whole-run figure: algorithmic bytes of every iteration of every system
    (bytes_model per inner iteration, plus one float64 residual pass per
    outer step) over the wall time of the run."""
    ach = byte_total / wall / 1e9 if wall > 0 else 0.0
    return {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": what,
            "algorithmic_bytes_total": byte_total, "wall_s": wall}


def run_bytes(m, n, nnz, iters, outer, f32):
    """Algorithmic bytes of one solve: its inner iterations plus, per outer
    step, the refinement residual b - A x (matrix once, x, b and r64)."""
    v = 4 if f32 else 8
    return (iters * bytes_model(m, n, nnz, f32)["iter"] +
            max(1, outer) * ((v + 4) * nnz + 4 * m + 8 * n + 16 * m))


def run_batch(args):
    """256 uneven systems, FP32 storage + FP64 refinement to 1e-8, one launch
    per phase over all unfinished systems.  Only systems that reach the
    tolerance (status OK and the true residual checked on the host) count as
    solves, in this arm and in the plain float64 baseline (every system
    solved alone, matrices created before the timed loop as in the batch)."""
    import numpy as np
    import paper_2207_07615_amd as plss
    t0 = time.perf_counter()
    data = _pool_map(_gen_batch, range(args.nsys))
    log(f"generated {len(data)} systems in {time.perf_counter() - t0:.1f}s, "
        f"nnz total {sum(d[0].nnz for d in data)}")
    tol = 1e-8
    h = plss.Handle(0)
    import torch
    mats = [plss.Matrix(h, A.row_ptr, A.col_idx, A.vals, shape=(A.m, A.n), storage="f32") for A, _, _ in data]
    # right-hand sides and solutions stay in HBM (device tensors) in the timed regions
    gpu = torch.device("cuda:0")
    bs = [torch.from_numpy(b).to(gpu) for _, b, _ in data]
    torch.cuda.synchronize()
    kw = dict(tol=tol, maxit=args.maxit_cap, refine=True, inner_tol=1e-4)
    plss.solve_batch(h, mats[:8], bs[:8], **kw)   # warm-up (code objects, workspace)
    plss.kernel_times(h)
    t1 = time.perf_counter()
    xs, infos = plss.solve_batch(h, mats, bs, timing=True, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t1
    kms, kn = plss.kernel_times(h)
    xs = [x.cpu().numpy() for x in xs]
    rr = [host_relres(d[0], d[1], x) for x, d in zip(xs, data)]
    ok = [i["status"] == 0 and r <= tol for i, r in zip(infos, rr)]
    errs = [float(np.linalg.norm(x - d[2]) / np.linalg.norm(d[2])) for x, d, c in zip(xs, data, ok) if c]
    tot_nnz = sum(d[0].nnz for d in data)
    byte_total = sum(run_bytes(d[0].m, d[0].n, d[0].nnz, i["iters"], i["outer_iters"], True)
                     for d, i in zip(data, infos))
    # the same batch after the library's autotuner picked each matrix's tile
    # widths by timing its plain products (per matrix, per direction)
    t_tune = time.perf_counter()
    tiles = [M.autotune() for M in mats]
    t_tune = time.perf_counter() - t_tune
    t1 = time.perf_counter()
    xs_t, infos_t = plss.solve_batch(h, mats, bs, **kw)
    torch.cuda.synchronize()
    wall_t = time.perf_counter() - t1
    ok_t = sum(1 for x, i, d in zip(xs_t, infos_t, data)
               if i["status"] == 0 and host_relres(d[0], d[1], x.cpu().numpy()) <= tol)
    del mats
    # one system at a time, plain float64 Algorithm 1 on the same GPU
    m64 = [plss.Matrix(h, A.row_ptr, A.col_idx, A.vals, shape=(A.m, A.n)) for A, _, _ in data]
    plss.solve(h, m64[0], bs[0], tol=tol, maxit=args.maxit_cap)
    t2 = time.perf_counter()
    res64 = [plss.solve(h, M64, b, tol=tol, maxit=args.maxit_cap)[:2] for M64, b in zip(m64, bs)]
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t2
    ok64 = [i["status"] == 0 and host_relres(d[0], d[1], x.cpu().numpy()) <= tol for (x, i), d in zip(res64, data)]
    del m64
    nok, nok64 = sum(ok), sum(ok64)
    return base_line(METRIC, nok / wall, "solves/s", 1, 0, wall, "f32+f64",
                     {"workload": f"batch: {len(data)} systems, m log-U[1e3,2e5], n=m*U(.5,1), 5-50 nnz/row, "
                                  "FP32 storage + FP64 refinement, tol 1e-8", "nnz_total": tot_nnz,
                      "maxit": args.maxit_cap, "tiles": "default widths (autotuned run below)"},
                     counted="solves with status OK and host-checked ||b - A x||/||b|| <= tol",
                     converged=nok, systems=len(data), max_rel_err_vs_xstar=max(errs) if errs else None,
                     iters_total=sum(i["iters"] for i in infos),
                     kernel_ms_total=dict(zip(["spmv", "spmvt", "step", "update"], kms)),
                     roofline=aggregate_roofline(byte_total, wall, "whole batch (all phases)"),
                     plain_fp64={"solves_per_s": nok64 / t_plain, "converged": nok64, "wall_s": t_plain,
                                 "how": "every system alone, float64 storage, same GPU"},
                     speedup_vs_plain_fp64=(nok / wall) / (nok64 / t_plain) if nok64 else None,
                     autotuned={"solves_per_s": ok_t / wall_t, "converged": ok_t, "wall_s": wall_t,
                                "tune_s": t_tune, "widths_a_t": {f"{a},{t}": tiles.count((a, t))
                                                                 for a, t in sorted(set(tiles))}})


def run_multi(args):
    """Shared 500,000 x 250,000 (20 nnz/row) with 32 right-hand sides, block
    products, FP32 storage + FP64 refinement to 1e-8."""
    import numpy as np
    import paper_2207_07615_amd as plss
    import plss_inputs as gen
    import torch
    A, B, X = gen.shared_multi_rhs(storage=np.float32)
    h = plss.Handle(0)
    M = plss.Matrix(h, A.row_ptr, A.col_idx, A.vals, shape=(A.m, A.n), storage="f32")
    # the right-hand sides (row c of B_d is column c: B_d.t() is the m x nrhs
    # block, column-major as the library takes it) and the solutions stay in HBM
    gpu = torch.device("cuda:0")
    B_d = torch.from_numpy(np.ascontiguousarray(B)).to(gpu)
    torch.cuda.synchronize()
    kw = dict(tol=1e-8, maxit=5000, refine=True, inner_tol=1e-4)
    for _ in range(args.warmup):
        plss.solve_multi(h, M, B_d.t(), **kw)
    plss.kernel_times(h)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        Xg, infos = plss.solve_multi(h, M, B_d.t(), timing=True, **kw)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    Xg = Xg.cpu().numpy()
    kms, kn = plss.kernel_times(h)
    nrhs = B.shape[0]
    # block bytes per iteration: matrix once for all columns (float32 values + int32 index)
    per_spmm = 8 * A.nnz + 4 * A.m + nrhs * 4 * (2 * A.m + A.n)
    avg = [kms[q] / max(1, kn[q]) for q in range(4)]
    ach = per_spmm / (avg[0] * 1e-3) / 1e9
    errs = [float(np.linalg.norm(Xg[:, c] - X[c]) / np.linalg.norm(X[c])) for c in range(nrhs)]
    # same right-hand sides one at a time, plain float64 Algorithm 1
    M64 = plss.Matrix(h, A.row_ptr, A.col_idx, A.vals, shape=(A.m, A.n))
    t1 = time.perf_counter()
    for c in range(4):
        plss.solve(h, M64, B_d[c], tol=1e-8, maxit=5000)
    torch.cuda.synchronize()
    t_plain = (time.perf_counter() - t1) / 4 * nrhs
    return base_line(METRIC, args.steps * nrhs / wall, "solves/s", args.steps, args.warmup, wall, "f32+f64",
                     {"workload": "multi: shared 500,000 x 250,000 CSR, 20 nnz/row, 32 RHS block, "
                                  "FP32 storage + FP64 refinement, tol 1e-8", "nnz": A.nnz, "nrhs": nrhs},
                     iters_per_rhs=sum(i["iters"] for i in infos) / nrhs,
                     max_rel_err_vs_xstar=max(errs), converged=sum(1 for i in infos if i["status"] == 0),
                     kernel_ms=dict(zip(["spmm", "spmmt", "step", "update"], avg)),
                     roofline={"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": ach / HBM_PEAK_GBS, "traffic": None, "kernel": "block product with A",
                               "algorithmic_bytes_per_launch": per_spmm},
                     plain_fp64_one_rhs_at_a_time_s=t_plain, speedup_vs_plain_fp64=t_plain / (wall / args.steps))


def run_serve(args):
    """Served stream: systems with Poisson arrivals, FP32 storage + FP64
    refinement under continuous batching, against plain per-system FP64.
    Only requests that reach their own tolerance (status OK and the true
    residual checked on the host) count as solves, in both arms."""
    import numpy as np
    import paper_2207_07615_amd as plss
    import plss_inputs as gen
    t0 = time.perf_counter()
    data = _pool_map(_gen_stream, range(args.nsys))
    log(f"generated {len(data)} systems in {time.perf_counter() - t0:.1f}s")
    h = plss.Handle(0)
    budget = 200 << 30

    def cap(s):
        return min(s.A.n + 1000, args.maxit_cap)

    def serve(arrivals):
        srv = plss.Server(h, hbm_budget_bytes=budget, max_slots=256)
        t_start = time.perf_counter()
        reqs = []
        for (s, A32, b32), ta in zip(data, arrivals):
            while time.perf_counter() - t_start < ta:
                time.sleep(0.0005)
            reqs.append(srv.submit(A32, b32, storage="f32", tol=s.tol, maxit=cap(s),
                                   refine=True, inner_tol=1e-4))
        pending = list(range(len(reqs)))
        got = {}
        while pending:
            nxt = []
            for i in pending:
                r = srv.poll(reqs[i])
                if r is None:
                    nxt.append(i)
                else:
                    got[i] = r
            pending = nxt
            time.sleep(0.0005)
        wall = time.perf_counter() - t_start
        srv.close()
        return wall, [got[i] for i in range(len(reqs))]

    def counted(res, which):
        out = []
        for (s, A32, b32), (x, info) in zip(data, res):
            A, b = (A32, b32) if which == "f32" else (s.A, s.b)
            out.append(info["status"] == 0 and host_relres(A, b, x) <= s.tol)
        return out

    def by_tol(flags):
        return {f"{t:g}": [sum(1 for (s, _, _), f in zip(data, flags) if s.tol == t and f),
                           sum(1 for s, _, _ in data if s.tol == t)] for t in (1e-6, 1e-10)}

    def pct(v, q):
        v = sorted(v)
        return v[min(len(v) - 1, max(0, int(math.ceil(q * len(v))) - 1))] if v else None

    n = len(data)
    serve([0.0] * min(n, 8))                     # warm-up (code objects, workspace)
    wall_sat, res_sat = serve([0.0] * n)
    ok_sat = counted(res_sat, "f32")
    rate = 0.7 * sum(ok_sat) / wall_sat
    arr = gen.poisson_arrivals(n, rate)
    wall_p, res_p = serve(list(arr))
    ok_p = counted(res_p, "f32")
    lat_ok = [info["ms"] for (_, info), f in zip(res_p, ok_p) if f]
    lat_all = [info["ms"] for _, info in res_p]
    byte_total = sum(run_bytes(s.A.m, s.A.n, s.A.nnz, info["iters"], info["outer_iters"], True)
                     for (s, _, _), (_, info) in zip(data, res_sat))
    # plain per-system FP64 Algorithm 1 on the same GPU, one request at a time
    # (each request brings its matrix: upload and transpose are timed, as in
    # the served arm)
    t1 = time.perf_counter()
    res64 = []
    for s, _, _ in data:
        M64 = plss.Matrix(h, s.A.row_ptr, s.A.col_idx, s.A.vals, shape=(s.A.m, s.A.n))
        res64.append(plss.solve(h, M64, s.b, tol=s.tol, maxit=cap(s))[:2])
        del M64
    t_plain = time.perf_counter() - t1
    ok64 = counted(res64, "f64")
    nsat, n64 = sum(ok_sat), sum(ok64)
    return base_line(METRIC, nsat / wall_sat, "solves/s", 1, 0, wall_sat, "f32+f64",
                     {"workload": f"serve: {n} systems of the stream recipe (m log-U[1e3,1e6], n/m U(.3,1), "
                                  "Zipf(1.5) rows clipped to [1,100], tol 1e-6 or 1e-10), FP32 + FP64 refinement, "
                                  "continuous batching", "nnz_total": sum(s.A.nnz for s, _, _ in data),
                      "maxit": f"min(n + 1000, {args.maxit_cap})"},
                     counted="requests with status OK and host-checked ||b - A x||/||b|| <= their tol",
                     systems=n, converged=nsat, converged_by_tol=by_tol(ok_sat),
                     saturated_solves_per_s=nsat / wall_sat, poisson_rate=rate,
                     poisson_solves_per_s=sum(ok_p) / wall_p, poisson_converged=sum(ok_p),
                     p50_ms=pct(lat_ok, 0.5), p99_ms=pct(lat_ok, 0.99),
                     p50_ms_all_requests=pct(lat_all, 0.5), p99_ms_all_requests=pct(lat_all, 0.99),
                     roofline=aggregate_roofline(byte_total, wall_sat, "whole saturated run (all phases)"),
                     plain_fp64={"solves_per_s": n64 / t_plain, "converged": n64, "wall_s": t_plain,
                                 "converged_by_tol": by_tol(ok64),
                                 "how": "every request alone (matrix upload + solve), float64, same GPU"},
                     speedup_vs_plain_fp64=(nsat / wall_sat) / (n64 / t_plain) if n64 else None)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--m", type=int, default=2_000_000)
    ap.add_argument("--n", type=int, default=500_000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle baseline")
    ap.add_argument("--no-fp32", action="store_true", help="skip the float32 + refinement arm")
    ap.add_argument("--no-w", action="store_true", help="skip the PLSS W arm (column-norm weights)")
    ap.add_argument("--no-rp", action="store_true", help="skip the randomized-projection arm")
    ap.add_argument("--no-pair", action="store_true", help="skip the fused residual-pair measurement")
    ap.add_argument("--autotune", action="store_true", help="pick tile widths by measurement")
    ap.add_argument("--layout", default="auto", choices=["auto", "tiles", "stripes"],
                    help="product layout of the large workload (auto: chosen from the shape)")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run a 1 GiB device copy (calibrates profiler byte counters)")
    ap.add_argument("--config", default="large",
                    choices=["large", "small", "underdet", "batch", "multi", "serve"])
    ap.add_argument("--nsys", type=int, default=0, help="systems for batch/serve (default 256 / 200)")
    ap.add_argument("--maxit-cap", type=int, default=4000,
                    help="batch/serve: iteration bound min(n + 1000, cap) per system")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.config != "large":
        if not args.nsys:
            args.nsys = 256 if args.config == "batch" else 200
        fn = {"small": run_small, "underdet": run_underdet, "batch": run_batch,
              "multi": run_multi, "serve": run_serve}[args.config]
        print(json.dumps(fn(args)), flush=True)
        return

    import numpy as np
    import torch

    import paper_2207_07615_amd as plss
    import plss_inputs as gen

    t0 = time.perf_counter()
    sysm = gen.large(m=args.m, n=args.n)
    A = sysm.A
    log(f"generated m={A.m} n={A.n} nnz={A.nnz} in {time.perf_counter() - t0:.1f}s")

    dev = torch.device("cuda:0")
    h = plss.Handle(0)
    t0 = time.perf_counter()
    M = plss.Matrix(h, A.row_ptr, A.col_idx, A.vals, shape=(A.m, A.n))
    log(f"device store (upload + CSC) in {time.perf_counter() - t0:.2f}s")
    if args.autotune:
        log(f"tile widths {M.autotune()}")
    if args.layout != "auto":
        on = args.layout == "stripes"
        M.layout(a_stripes=on, t_stripes=on)
    layout = M.layout()
    log(f"layout {layout}")
    b = torch.from_numpy(sysm.b).to(dev)
    torch.cuda.synchronize()

    kw = dict(tol=1e-8, maxit=1000)
    for _ in range(args.warmup):
        plss.solve(h, M, b, **kw)
    plss.kernel_times(h)  # reset
    torch.cuda.synchronize()
    lat, iters = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        x, info, _ = plss.solve(h, M, b, timing=True, **kw)
        lat.append(time.perf_counter() - ts)
        iters.append(info["iters"])
        assert info["status"] == 0, info
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    kms, kn = plss.kernel_times(h)
    relres_true = info["relres_true"]
    if args.calib_copy:
        # an elementwise kernel that reads 1 GiB and writes 1 GiB
        src = torch.ones(1 << 27, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.mul(src, 2.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    err_xstar = float(torch.linalg.norm(x - torch.from_numpy(sysm.xstar).to(dev)) /
                      np.linalg.norm(sysm.xstar))

    bm = bytes_model(A.m, A.n, A.nnz)
    lay_name = ("stripes" if layout["a_stripes"] and layout["t_stripes"]
                else "tiles" if not (layout["a_stripes"] or layout["t_stripes"]) else "mixed")
    tot_iters = sum(iters)
    iters_per_s = tot_iters / wall
    avg = [kms[q] / max(1, kn[q]) for q in range(4)]
    dom = 0 if avg[0] >= avg[1] else 1
    dom_bytes = bm["spmv"] if dom == 0 else bm["spmvt"]
    achieved = dom_bytes / (avg[dom] * 1e-3) / 1e9
    pair_gbs = (bm["spmv"] + bm["spmvt"]) / ((avg[0] + avg[1]) * 1e-3) / 1e9
    lat_ms = sorted(1e3 * v for v in lat)

    out = {
        "metric": METRIC,
        "value": iters_per_s,
        "unit": "iters/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * wall / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (seeded; stands in for the paper's SuiteSparse matrices)",
        "config": {"workload": "large: 2,000,000 x 500,000 CSR, Zipf(1.5) rows clipped to [2,2000], "
                               "N(0,1), residual sketch, FP64, rel. tol 1e-8",
                   "m": A.m, "n": A.n, "nnz": A.nnz, "tol": 1e-8, "maxit": 1000,
                   "layout": layout},
        "iters_per_solve": tot_iters / args.steps,
        "solves_per_s": args.steps / wall,
        "p50_ms": lat_ms[len(lat_ms) // 2],
        "p99_ms": lat_ms[min(len(lat_ms) - 1, int(math.ceil(0.99 * len(lat_ms))) - 1)],
        "hbm_gbps_iteration": bm["iter"] * iters_per_s / 1e9,
        "hbm_gbps_spmv_pair": pair_gbs,
        "kernel_ms": {"spmv": avg[0], "spmvt": avg[1], "blocksum_step": avg[2], "update": avg[3]},
        "relres_true": relres_true,
        "rel_err_vs_xstar": err_xstar,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": recorded_traffic(dom, lay_name),
                     "traffic_source": ("recorded: calibrated rocprofv3 FETCH_SIZE / WRITE_SIZE passes of this "
                                        "kernel (profiles/large_fp64_traffic.txt), reported only while the "
                                        "kernel sources and the layout match those the counters were taken "
                                        "with; not measured in this run"),
                     "kernel": (("k_sspmv RESID" if layout["a_stripes"] else "k_spmv RESID") +
                                " (r -= A p, partial rho)") if dom == 0 else
                               (("k_sspmv TRANSB (row-block products A_b^T r_b)" if layout["t_stripes"]
                                 else "k_spmv TRANS (y = A^T r)")),
                     "algorithmic_bytes_per_launch": dom_bytes},
    }

    if not args.no_fp32:
        A32 = A.astype(np.float32)
        b32 = torch.from_numpy(gen.rhs(A32, sysm.xstar)).to(dev)
        M32 = plss.Matrix(h, A.row_ptr, A.col_idx, A.vals, shape=(A.m, A.n), storage="f32")
        if args.autotune:
            M32.autotune()
        if args.layout != "auto":
            on = args.layout == "stripes"
            M32.layout(a_stripes=on, t_stripes=on)
        kw32 = dict(tol=1e-8, maxit=4000, refine=True, inner_tol=1e-4, max_outer=20)
        plss.solve(h, M32, b32, **kw32)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        n32 = max(1, args.steps // 2)
        its32 = []
        for _ in range(n32):
            x32, i32, _ = plss.solve(h, M32, b32, **kw32)
            its32.append(i32["iters"])
        torch.cuda.synchronize()
        w32 = time.perf_counter() - t1
        out["fp32_refine"] = {
            "solves_per_s": n32 / w32, "ms_per_solve": 1e3 * w32 / n32,
            "iters_per_solve": sum(its32) / n32, "outer_iters": i32["outer_iters"],
            "relres_true": i32["relres_true"], "status": i32["status_name"],
            "speedup_vs_fp64_solves": (n32 / w32) / (args.steps / wall),
            "iters_per_s": sum(its32) / w32,
            "hbm_gbps_iteration": bytes_model(A.m, A.n, A.nnz, True)["iter"] * sum(its32) / w32 / 1e9,
            "layout": M32.layout(),
        }
        del M32

    if not args.no_w:
        # PLSS W (Section 4.1): W = diag(1/||A_{:,j}||); the weights stream
        # twice more per iteration (the block sum's phi and the update)
        wi_h = np.sqrt(np.bincount(A.col_idx, weights=A.vals.astype(np.float64) ** 2, minlength=A.n))
        wi = torch.from_numpy(np.where(wi_h > 0, wi_h, 1.0)).to(dev)
        kww = dict(tol=1e-8, maxit=1000, wi=wi)
        plss.solve(h, M, b, **kww)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        nw = max(1, args.steps // 2)
        itsw = []
        for _ in range(nw):
            xw, iw, _ = plss.solve(h, M, b, **kww)
            itsw.append(iw["iters"])
        torch.cuda.synchronize()
        ww = time.perf_counter() - t1
        out["plss_w"] = {
            "solves_per_s": nw / ww, "ms_per_solve": 1e3 * ww / nw,
            "iters_per_solve": sum(itsw) / nw, "iters_per_s": sum(itsw) / ww,
            "relres_true": iw["relres_true"], "status": iw["status_name"],
            "solves_per_s_vs_plain": (nw / ww) / (args.steps / wall),
        }

    if not args.no_rp:
        # the paper's randomized projection (fresh 5-column Gaussian sketch per
        # iteration, r = 5 for n > 1e5 as in Experiment III) for a fixed number
        # of iterations, against Algorithm 1 after as many iterations
        krp = 100
        kwr = dict(sketch="randproj", block=5, seed=761512, tol=1e-300, maxit=krp)
        plss.solve(h, M, b, **dict(kwr, maxit=2))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xr, ir, _ = plss.solve(h, M, b, **kwr)
        torch.cuda.synchronize()
        wr = time.perf_counter() - t1
        xp, ip, _ = plss.solve(h, M, b, tol=1e-300, maxit=krp)
        out["randproj_r5"] = {
            "iters": ir["iters"], "iters_per_s": ir["iters"] / wr, "ms_per_iter": 1e3 * wr / ir["iters"],
            "relres_true_after": ir["relres_true"], "plss_relres_true_after_same_iters": ip["relres_true"],
        }

    if not args.no_pair:
        # the fused residual pair (one pass over the CSR, two-level sum for y)
        # against the iteration's own products (both products, the block sum
        # and the step scalars, from the timed solves above)
        rng = np.random.default_rng(17)
        pd = torch.from_numpy(rng.standard_normal(A.n)).to(dev)
        rd = torch.from_numpy(rng.standard_normal(A.m)).to(dev)
        plss.residual_pair(h, M, pd, rd)  # builds the position map
        torch.cuda.synchronize()
        npair = 10
        t1 = time.perf_counter()
        for _ in range(npair):
            plss.residual_pair(h, M, pd, rd)
        torch.cuda.synchronize()
        wp = (time.perf_counter() - t1) / npair
        pair_bytes = 32 * A.nnz + 20 * A.m + 20 * A.n
        ref_ms = avg[0] + avg[1] + avg[2]
        out["residual_pair"] = {
            "ms_per_call": 1e3 * wp, "how": "host wall per call on device tensors (includes the call's sync)",
            "bytes_per_call": pair_bytes, "gbps": pair_bytes / wp / 1e9,
            "iteration_products_ms": ref_ms, "ratio_vs_iteration_products": 1e3 * wp / ref_ms,
        }

    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(sysm)
        # the same oracle with every host thread pool at the machine's CPU share
        out["cpu_baseline_all_cores"] = cpu_baseline(sysm, iters=40, threads=min(16, os.cpu_count() or 1))

    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
