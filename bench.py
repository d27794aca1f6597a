#!/usr/bin/env python3
"""Benchmark of the gridding hot path on one MI355X.

One step = the whole path over one batch of 2M synthetic multibeam soundings
already resident in HBM:
    bin (rebase + counting sort)  ->  IDW p=2 r=6 m k=16 with the nearest pick
    on the 4096^2 grid at 2 m     ->  bilinear 2x resample to 8192^2 at 1 m.
`value` = grid nodes of the 4096^2 IDW grid per second of step time.

Prints ONE JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import gc
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "IDW grid nodes/s at 2M soundings→4096²; p99 ping-to-grid latency vs plain"
HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_threads() -> int:
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return len(os.sched_getaffinity(0))


# Sources that define each profiled kernel (its code and its argument structs).
KERNEL_SOURCES = {
    "k_idw_window": ["idw_window_impl.hpp", "idw_window.hip", "auv_internal.hpp"],
    "k_bilinear": ["bilinear_kernels.hip", "resample_axis.hpp", "auv_internal.hpp"],
    "k_kriging": ["kriging.hip", "resample_axis.hpp", "auv_internal.hpp"],
    "k_bicubic": ["bilinear_kernels.hip", "resample_axis.hpp", "auv_internal.hpp"],
}


def kernel_source_digest(kernel: str) -> str:
    """Digest of the HIP sources of `kernel`, to tell whether a committed counter
    profile still describes the kernel being timed."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2505_22675_amd", "csrc")
    for fn in KERNEL_SOURCES[kernel]:
        with open(os.path.join(csrc, fn), "rb") as f:
            h.update(fn.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


VALU_ISSUE_PEAK = 256 * 4 * 2.4e9 / 4   # wave64 VALU instructions per second (16-lane SIMDs)


def valu_from_profile(kernel: str):
    """VALU wave instructions per launch of `kernel` from the committed
    rocprofv3 SQ summary; None when there is none or the sources changed."""
    path = os.path.join(ROOT, "profiles", "valu_issue_swath2M.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("valu_instr "):
                _, name, val, digest = line.split()
                rec[name] = (int(val), digest)
    if kernel not in rec or rec[kernel][1] != kernel_source_digest(kernel):
        return None
    return rec[kernel][0]


LANE_OPS_PEAK = 256 * 4 * 16 * 2.4e9    # FP32/INT32 lane operations per second, not packed
ALU_OPS_PER_PAIR = 10                    # exact D^2 (4 mul, 2 add), compare, weight, 2 accumulates


def profile_source(fname: str, kernel: str) -> str:
    return f"profiles/{fname} (sources digest {kernel_source_digest(kernel)})"


def traffic_from_profile(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel calibration).
    None when there is no summary or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_swath2M.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as f:
        for line in f:
            if line.startswith("traffic_bytes "):
                _, name, val, digest = line.split()
                rec[name] = (int(val), digest)
    if kernel not in rec or rec[kernel][1] != kernel_source_digest(kernel):
        return None
    return rec[kernel][0]


def cpu_baseline(s, up_desc, nodes):
    """The FP64 oracle timed on the host's cores over the same step (binned IDW
    + nearest on every node, then the bilinear 2x), repeated until at least 10 s
    of CPU work has run; value = grid nodes per second of the mean repetition."""
    import oracle
    oracle.build(force=False)
    th = host_threads()
    og = oracle.Grid(s.grid.x0, s.grid.y0, s.grid.dx, s.grid.dy, s.grid.nx, s.grid.ny)
    ug = oracle.Grid(up_desc.x0, up_desc.y0, up_desc.dx, up_desc.dy, up_desc.nx, up_desc.ny)
    log(f"cpu baseline: FP64 oracle, binned search, {th} threads, full grid")
    reps, t_idw, t_bil = 0, 0.0, 0.0
    while reps < 200 and (t_idw + t_bil < 10.0 or reps == 0):
        c0 = time.perf_counter()
        oz, _, _ = oracle.idw(og, s.x, s.y, s.z, s.radius, s.power, s.min_pts, s.max_pts,
                              bin_log2=19, nthreads=th)
        c1 = time.perf_counter()
        oracle.bilinear(og, oz, ug, nthreads=th)
        c2 = time.perf_counter()
        t_idw += c1 - c0
        t_bil += c2 - c1
        reps += 1
    per = (t_idw + t_bil) / reps
    out = {"value": round(nodes / per, 1), "unit": "grid nodes/s", "cores": th,
           "kind": "oracle",
           "sample": f"the full step repeated {reps} times ({t_idw + t_bil:.1f} s): binned "
                     f"FP64 IDW+nearest on all {nodes} nodes ({t_idw / reps:.3f} s each) + "
                     f"bilinear to 8192^2 ({t_bil / reps:.3f} s each)"}
    log(f"cpu baseline {out['value']:.3e} nodes/s over {reps} repetitions")
    # brute force (every sounding tested at every node) on seeded sampled nodes
    import numpy as np
    sample = np.random.default_rng(2).choice(nodes, 16384, replace=False).astype(np.int64)
    c0 = time.perf_counter()
    oracle.idw(og, s.x, s.y, s.z, s.radius, s.power, s.min_pts, s.max_pts, bin_log2=-1,
               nodes=sample, nthreads=th)
    t_bf = time.perf_counter() - c0
    out["brute_force_sample"] = {"nodes": int(sample.size), "seconds": round(t_bf, 3),
                                 "pair_tests": int(sample.size) * int(s.n),
                                 "nodes_per_s": round(sample.size / t_bf, 1)}
    out["host"] = {"cpus": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
                   "model": cpu_model()}
    log(f"cpu brute force: {sample.size} nodes in {t_bf:.2f} s")
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _median_ms(fn, stream, reps):
    """Median HIP-event time of fn() on stream over reps launches (after two
    untimed ones)."""
    import numpy as np
    import torch
    fn()
    fn()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for e0, e1 in evs:
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    return float(np.median([e0.elapsed_time(e1) for e0, e1 in evs]))


def _cpu_median_ms(fn):
    """Median wall time of fn() in ms over up to five runs (fewer once a second
    has been spent; at least one), after untimed runs (up to 20, or 0.2 s) that
    start and settle the host thread pool."""
    w0 = time.perf_counter()
    for _ in range(20):
        fn()
        if time.perf_counter() - w0 > 0.2:
            break
    times = []
    while len(times) < 5 and (not times or sum(times) < 1.0):
        c0 = time.perf_counter()
        fn()
        times.append(time.perf_counter() - c0)
    return round(statistics.median(times) * 1e3, 3)


GRID_A_POINTS = [10 ** 3, 10 ** 4, 10 ** 5, 10 ** 6, 10 ** 7, 10 ** 8]
GRID_A_CPU_MAX = 10 ** 6
RESAMPLERS = ("bilinear", "bicubic", "kriging")


def cpu_grid_a(s, v, d, range_m):
    """Oracle leg of the grid-A sweep: median ms of each resampler."""
    import oracle
    oracle.build(force=False)
    th = host_threads()
    og = oracle.Grid(s.x0, s.y0, s.dx, s.dy, s.nx, s.ny)
    od = oracle.Grid(d.x0, d.y0, d.dx, d.dy, d.nx, d.ny)
    src = v.astype("float64")
    out = {}
    for m in RESAMPLERS:
        if m == "kriging":
            fn = lambda: oracle.kriging(og, src, od, range_m, nthreads=th)
        else:
            fn = lambda: getattr(oracle, m)(og, src, od, nthreads=th)
        out[f"cpu_{m}_ms"] = _cpu_median_ms(fn)
    return out


def grid_a_sweep(ag, dev, with_cpu):
    """Row infill (grid A) from 1e3 to 1e8 interpolated nodes: median kernel
    time of each resampler, and the oracle's time up to 1e6 nodes."""
    import torch
    from gen import grid_a_case
    stream = torch.cuda.current_stream()
    rows = []
    for pts in GRID_A_POINTS:
        s, v, d = grid_a_case(pts)
        src = torch.from_numpy(v).to(dev)
        dst = torch.empty((d.ny, d.nx), dtype=torch.float32, device=dev)
        rm = 3.0 * s.dx
        fns = {
            "bilinear": lambda: ag.auv_resample_bilinear(src, s, dst, d, stream=stream),
            "bicubic": lambda: ag.auv_resample_bicubic(src, s, dst, d, stream=stream),
            "kriging": lambda: ag.auv_resample_kriging(src, s, dst, d, rm, stream=stream),
        }
        row = {"points": d.nx * d.ny, "src": [s.nx, s.ny]}
        for m in RESAMPLERS:
            row[f"gpu_{m}_ms"] = round(_median_ms(fns[m], stream, 20 if pts <= 10 ** 7 else 5), 5)
        if with_cpu and pts <= GRID_A_CPU_MAX:
            row.update(cpu_grid_a(s, v, d, rm))
        rows.append(row)
        log("grid A " + " ".join(f"{k}={v}" for k, v in row.items()))
        del src, dst
    return {"workload": "rows filled midway between the rows of a fractal-seafloor grid "
                        "(1 m nodes), bilinear / Catmull-Rom / kriging (range 3 m)",
            "rows": rows}


def _fill_metrics(est, truth, interp):
    import numpy as np
    v = est[interp].astype(np.float64)
    t = truth[interp]
    ok = ~np.isnan(v)
    e = v[ok] - t[ok]
    return {"holes": int((~ok).sum()), "mae": round(float(np.abs(e).mean()), 5),
            "rmse": round(float(np.sqrt((e * e).mean())), 5)}


def grid_b_report(ag, dev, with_cpu, n_fine=2048):
    """Random-removal infill (grid B) on a 2048^2 fractal-seafloor truth at
    4 m: every other node recorded, 1 %, 5 % and 10 % of those removed, every
    unrecorded node filled by the three resamplers (recorded grid -> fine grid)
    and by the scattered path (bin + IDW p=2, r=12 m, of the recorded nodes);
    MAE / RMSE against the truth with holes excluded and counted, and the
    kernel time of each fill.  The oracle's time of each fill is added at 5 %."""
    import torch
    from gen import grid_b_case
    stream = torch.cuda.current_stream()
    log(f"grid B: sampling the {n_fine}^2 truth")
    base = grid_b_case(n_fine, 0.0)
    out = {"workload": f"{n_fine}^2 fractal seafloor at 4 m, every other node recorded, "
                       "random removal of recorded nodes; fills: bilinear, Catmull-Rom, "
                       "kriging (range 24 m, and the range fitted to the recorded grid's "
                       "semivariogram) from the recorded grid, IDW p=2 r=12 m from the "
                       "recorded nodes", "cases": []}
    for frac in (0.01, 0.05, 0.1):
        c = grid_b_case(n_fine, frac, truth=base["truth"])
        cs, ts = c["coarse_spec"], c["truth_spec"]
        coarse = torch.from_numpy(c["coarse"]).to(dev)
        fine = torch.empty((ts.ny, ts.nx), dtype=torch.float32, device=dev)
        rm = 3.0 * cs.dx
        radius = 3.0 * ts.dx
        grid = ag.auv_grid_create(ts)
        x, y, z = (torch.from_numpy(c[k]).to(dev) for k in ("x", "y", "z"))
        ws = torch.empty(ag.auv_bin_workspace_size(grid, int(x.numel()), radius, 0),
                         dtype=torch.uint8, device=dev)
        params = ag.idw_params(2.0, radius, 1, 0)

        def idw():
            bins = ag.auv_bin_points(grid, x, y, z, radius, 0, ws=ws, stream=stream)
            ag.auv_interp_idw(grid, bins, params, fine, None, None, None, stream=stream)

        # the kriging range fitted to the recorded grid: its semivariogram
        # along the axes at lags 1..16 (8..128 m), exponential model
        t0 = time.perf_counter()
        fit_range, fit_sill, fit_rc = ag.fit_variogram_range(coarse, cs, 64, stream=stream)
        fit_ms = (time.perf_counter() - t0) * 1e3
        if fit_rc != ag.AUV_OK:
            fit_range = rm
        fns = {
            "bilinear": lambda: ag.auv_resample_bilinear(coarse, cs, fine, ts, stream=stream),
            "bicubic": lambda: ag.auv_resample_bicubic(coarse, cs, fine, ts, stream=stream),
            "kriging": lambda: ag.auv_resample_kriging(coarse, cs, fine, ts, rm, stream=stream),
            "kriging_fitted": lambda: ag.auv_resample_kriging(coarse, cs, fine, ts, fit_range,
                                                              stream=stream),
            "idw": idw,
        }
        case = {"removal": frac, "recorded": int(x.numel()),
                "interpolated": int(c["interp"].sum()),
                "variogram_fit": {"range_m": round(fit_range, 3), "sill_m2": round(fit_sill, 3),
                                  "status": int(fit_rc), "lags": 64,
                                  "host_ms_incl_gpu": round(fit_ms, 3)},
                "methods": {}}
        for m, fn in fns.items():
            ms = _median_ms(fn, stream, 20)
            fn()
            torch.cuda.synchronize()
            r = _fill_metrics(fine.cpu().numpy(), c["truth"], c["interp"])
            r["gpu_ms"] = round(ms, 5)
            case["methods"][m] = r
        if with_cpu and frac == 0.05:
            for m, ms in cpu_grid_b(c, rm, radius).items():
                case["methods"][m]["cpu_ms"] = ms
        out["cases"].append(case)
        log(f"grid B {frac}: " + "; ".join(
            f"{m} mae={r['mae']} rmse={r['rmse']} holes={r['holes']} {r['gpu_ms']} ms"
            for m, r in case["methods"].items()))
        ag.auv_grid_destroy(grid)
    return out


def cpu_grid_b(c, range_m, radius):
    """Oracle leg of the grid-B protocol: median ms of each fill."""
    import oracle
    oracle.build(force=False)
    th = host_threads()
    cs, ts = c["coarse_spec"], c["truth_spec"]
    oc = oracle.Grid(cs.x0, cs.y0, cs.dx, cs.dy, cs.nx, cs.ny)
    ot = oracle.Grid(ts.x0, ts.y0, ts.dx, ts.dy, ts.nx, ts.ny)
    src = c["coarse"].astype("float64")
    out = {}
    for m in RESAMPLERS + ("idw",):
        if m == "kriging":
            fn = lambda: oracle.kriging(oc, src, ot, range_m, nthreads=th)
        elif m == "idw":
            fn = lambda: oracle.idw(ot, c["x"], c["y"], c["z"], radius, 2.0, 1, 0,
                                    bin_log2=19, nthreads=th)
        else:
            fn = lambda: getattr(oracle, m)(oc, src, ot, nthreads=th)
        out[m] = _cpu_median_ms(fn)
    return out


def precision_report(ag, dev):
    """The same swath at UTM-scale coordinates (easting 5e5, northing 4e6): each
    precision variant of the IDW against the FP64 oracle, plus its kernel time."""
    import numpy as np
    import torch

    import oracle
    from gen import workload_cfg4

    log("precision variants on UTM-scale coordinates")
    s = workload_cfg4()
    og = oracle.Grid(s.grid.x0, s.grid.y0, s.grid.dx, s.grid.dy, s.grid.nx, s.grid.ny)
    oz, oc, onn = oracle.idw(og, s.x, s.y, s.z, s.radius, s.power, s.min_pts, s.max_pts,
                             bin_log2=19, nthreads=host_threads())
    grid = ag.auv_grid_create(s.grid)
    x, y, z = (torch.from_numpy(a).to(dev) for a in (s.x, s.y, s.z))
    bins = ag.auv_bin_points(grid, x, y, z, s.radius, 0)
    out = {}
    names = {ag.AUV_P_FP32_REBASE: "fp64_rebase_fp32", ag.AUV_P_FP16_OFFSETS: "fp16_offsets",
             ag.AUV_P_FP32_ABSOLUTE: "fp32_absolute"}
    for prec, name in names.items():
        res = ag.grid_idw(grid, bins, power=s.power, min_pts=s.min_pts, max_pts=s.max_pts,
                          with_counts=True, with_nearest=True, precision=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            ag.grid_idw(grid, bins, power=s.power, min_pts=s.min_pts, max_pts=s.max_pts,
                        with_counts=True, precision=prec)
        e1.record()
        torch.cuda.synchronize()
        gz = res["z"].cpu().numpy().astype(np.float64)
        gc = res["cnt"].cpu().numpy()
        gn = res["nn_idx"].cpu().numpy()
        both = ~np.isnan(gz) & ~np.isnan(oz)
        err = np.abs(gz[both] - oz[both])
        rel = err / np.abs(oz[both])
        # nodes whose neighbour set matches the oracle's (same count and same
        # nearest member): their error is the variant's arithmetic; the rest
        # flipped a member across the radius or reordered the nearest
        same = (gc == oc) & (gn == onn)
        sm = same[both]

        def stats(e):
            return ({"nodes": int(e.size), "max_abs_m": float(e.max()),
                     "rms_m": float(np.sqrt((e ** 2).mean()))} if e.size else {"nodes": 0})
        out[name] = {"max_abs_m": float(err.max()), "rms_m": float(np.sqrt((err ** 2).mean())),
                     "max_rel": float(rel.max()),
                     "nan_mask_mismatch": int((np.isnan(gz) != np.isnan(oz)).sum()),
                     "count_mismatch": int((gc != oc).sum()),
                     "same_neighbours": stats(err[sm]), "flipped_neighbours": stats(err[~sm]),
                     "idw_ms": round(e0.elapsed_time(e1) / 5, 4)}
        log(f"  {name}: {out[name]}")
    return out


def batched_report(ag, dev, reps=20, with_plain=True, tune_in=None, tune_out=None):
    """256 uneven tiles (1e3..2e5 soundings, 64^2..1024^2 nodes, p in {1,2,3}):
    the plain form (tile after tile, default bin size and kernel choice, no
    graph) against the batched form (autotuned per tile class, batched
    binning, persistent kernels, one HIP graph)."""
    import tempfile

    import numpy as np
    import torch

    from gen import checksum, workload_cfg3_tiles

    log("generating 256-tile batched workload")
    tiles = workload_cfg3_tiles()
    keep, items = [], []
    n_pts = n_nodes = 0
    for s in tiles:
        x, y, z = (torch.from_numpy(a).to(dev) for a in (s.x, s.y, s.z))
        shape = (s.grid.ny, s.grid.nx)
        zo = torch.empty(shape, dtype=torch.float32, device=dev)
        no = torch.empty(shape, dtype=torch.int32, device=dev)
        nz = torch.empty(shape, dtype=torch.float32, device=dev)
        desc = ag.make_desc(s.grid.x0, s.grid.y0, s.grid.dx, s.grid.dy, s.grid.nx, s.grid.ny)
        p = ag.idw_params(s.power, s.radius, s.min_pts, s.max_pts)
        items.append(ag.batch_item(desc, x, y, z, p, zo, None, no, nz))
        keep.append((x, y, z, zo, no, nz))
        n_pts += s.n
        n_nodes += s.grid.nx * s.grid.ny
    plain = ag.Batch(items)
    with tempfile.TemporaryDirectory() as td:
        if tune_in:
            # a table from an earlier run (counter passes: timing candidates
            # under a profiler would pick from distorted times)
            path, tune_s = tune_in, None
        else:
            path = os.path.join(td, "tune.txt")
            t0 = time.perf_counter()
            ag.auv_batch_autotune(items, plain.ws, path)
            tune_s = time.perf_counter() - t0
        tuned = ag.Batch(items, tune_path=path)
        table = [ln.strip() for ln in open(path) if ln.startswith("class ")]
        if tune_out:
            with open(tune_out, "w") as f:
                f.write("\n".join(table) + "\n")
    plans = [tuned.item_plan(i) for i in range(len(items))]

    def timed(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(reps)]
        for e0, e1 in evs:
            e0.record()
            fn()
            e1.record()
        torch.cuda.synchronize()
        ms = np.array([e0.elapsed_time(e1) for e0, e1 in evs])
        return float(np.median(ms)), float(ms.min())

    plain_med, plain_min = timed(plain.launch_plain) if with_plain else (float("nan"),) * 2
    batch_med, batch_min = timed(tuned.launch)
    # selected pairs of every tile (per-item IDW with counts, after timing)
    pairs = {"dense": 0, "sparse": 0}
    for k, s_ in enumerate(tiles):
        g_ = ag.auv_grid_create(s_.grid)
        x_, y_, z_ = keep[k][:3]
        b_ = ag.auv_bin_points(g_, x_, y_, z_, s_.radius, 0)
        r_ = ag.grid_idw(g_, b_, power=s_.power, min_pts=s_.min_pts, max_pts=s_.max_pts,
                         with_counts=True)
        form = "dense" if plans[k][1] == ag.AUV_ALGO_DENSE else "sparse"
        pairs[form] += int(r_["cnt"].sum(dtype=torch.int64).item())
        del r_, b_
    log(f"batched workload: plain {plain_med:.3f} ms, batched {batch_med:.3f} ms "
        f"(median of {reps})")
    alg_bytes = n_pts * 24 + n_nodes * 12
    out = {
        "workload": "256 uneven tiles: soundings log-uniform 1e3..2e5, side in "
                    "{64..1024} @ 2 m, p in {1,2,3}, r=6 m, k=16, min 1; IDW + nearest",
        "soundings": int(n_pts), "nodes": int(n_nodes),
        "input_sha": checksum(*[a for s in tiles for a in (s.x, s.y, s.z)]),
        "plain_ms": round(plain_med, 4) if with_plain else None,
        "plain_min_ms": round(plain_min, 4) if with_plain else None,
        "batched_ms": round(batch_med, 4), "batched_min_ms": round(batch_min, 4),
        "speedup": round(plain_med / batch_med, 3) if with_plain else None,
        "plain_nodes_per_s": round(n_nodes / (plain_med * 1e-3), 1) if with_plain else None,
        "batched_nodes_per_s": round(n_nodes / (batch_med * 1e-3), 1),
        "batched_hbm_frac": round(alg_bytes / (batch_med * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
        "selected_pairs": pairs,
        "batched_alu_frac": round(sum(pairs.values()) * ALU_OPS_PER_PAIR / (batch_med * 1e-3)
                                  / LANE_OPS_PEAK, 4),
        "algorithmic_bytes": int(alg_bytes),
        "autotune_s": round(tune_s, 2) if tune_s is not None else None, "tune_table": table,
        "dense_tiles": int(sum(a == ag.AUV_ALGO_DENSE for _, a in plans)),
    }
    plain.close()
    tuned.close()
    del keep
    return out


def serving_schedule_for_bench(duration):
    """The serving requests, generated before the GPU is touched (the vehicles
    are generated in forked worker processes)."""
    from gen import serving_schedule

    workers = max(1, min(16, os.cpu_count() or 1))
    log(f"generating {duration:.0f} s of serving requests ({workers} workers)")
    t = time.perf_counter()
    sched = serving_schedule(duration=duration, workers=workers)
    log(f"serving requests ready: {len(sched[1])} in {time.perf_counter() - t:.1f} s")
    return sched


def serving_report(ag, dev, sched, duration, stress=10.0):
    """16 vehicles (2048^2 grids at 2 m), Poisson requests at 20 Hz per vehicle
    of 2k..50k soundings (a +-60 deg fan at 150 m altitude), replayed in real
    time: FIFO (one request at a time) against continuous batching, at the
    nominal rate (the whole schedule, `duration` seconds) and at `stress`
    times the rate (the same schedule with its arrival times divided, lasting
    duration / stress seconds).  Latency = completion seen by the session -
    scheduled arrival.  `launches` counts the distinct launches the requests
    went in (a launch takes at most one request per vehicle)."""
    import numpy as np
    import torch

    grids, reqs = sched
    n_req = len(reqs)
    n_snd = int(sum(len(r.x) for r in reqs))
    out = {"workload": f"16 vehicles, 2048^2 grids @ 2 m, Poisson 20 Hz each, 2k..50k "
                       f"soundings per request, r=6 m p=2 no cap; {duration:.0f} s replay at "
                       f"the nominal rate, the same schedule at {stress:.0f}x its rate "
                       f"({duration / stress:.0f} s)",
           "requests": n_req, "soundings": n_snd}
    for mode, name in ((ag.AUV_SERVE_FIFO, "fifo"), (ag.AUV_SERVE_BATCHED, "batched")):
        for scale in (1.0, stress):
            desc = ag.session_desc(grids, power=2.0, radius=6.0, min_pts=1, max_request=50000,
                                   slots=64, mode=mode, z_ref=[-5000.0] * len(grids))
            fixed, per_v = ag.auv_session_budget(desc)
            arena = torch.empty(fixed + len(grids) * per_v, dtype=torch.uint8, device=dev)
            sess = ag.Session(desc, arena)
            empty = np.zeros(0)
            for v in range(len(grids)):      # admit every vehicle, load the kernels
                sess.submit(v, empty, empty, empty)
            sess.drain()
            # no collector pauses inside the replay: latency runs from each
            # request's scheduled arrival, so a stalled submit loop would count
            gc.collect()
            gc.disable()
            t0 = sess.now() + 0.05
            tickets = []
            plays = reqs
            for r in plays:
                ta = t0 + r.t_arrival / scale
                while True:
                    d = ta - sess.now()
                    if d <= 0:
                        break
                    if d > 2e-3:
                        time.sleep(d - 1e-3)
                tickets.append(sess.submit(r.vehicle, r.x, r.y, r.z, t_arrival=ta))
            sess.drain()
            gc.enable()
            infos = [sess.poll(t) for t in tickets]
            lat = np.array([i.t_done - i.t_arrival for i in infos]) * 1e3
            queue = np.array([i.t_launch - i.t_arrival for i in infos]) * 1e3
            launches = len({i.t_launch for i in infos})
            late = max(i.t_done for i in infos) - t0
            updates = 0
            for v in range(len(grids)):
                _, c = sess.read_grid(v)
                updates += int(c.sum().item())
            sess.close()
            del arena
            key = f"{name}_x{int(scale)}"
            out[key] = {"p50_ms": round(float(np.percentile(lat, 50)), 4),
                        "p99_ms": round(float(np.percentile(lat, 99)), 4),
                        "max_ms": round(float(lat.max()), 4),
                        "queue_p99_ms": round(float(np.percentile(queue, 99)), 4),
                        "node_updates": updates,
                        "node_updates_per_s": round(updates / late, 1),
                        "requests": len(plays),
                        "launches": launches,
                        "requests_per_launch": round(len(plays) / max(launches, 1), 3),
                        "soundings_per_s": round(n_snd / late, 1)}
            log(f"serving {key}: {len(plays)} requests, p50 {out[key]['p50_ms']:.3f} ms, "
                f"p99 {out[key]['p99_ms']:.3f} ms, max {out[key]['max_ms']:.3f} ms")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the UTM-scale precision-variant error report")
    ap.add_argument("--no-batched", action="store_true",
                    help="skip the 256-tile plain-vs-batched comparison")
    ap.add_argument("--batch-tune", default=None,
                    help="take the batched form's tune table from this file instead of autotuning")
    ap.add_argument("--save-batch-tune", default=None,
                    help="write the batched form's tune table to this file")
    ap.add_argument("--no-plain-batch", action="store_true",
                    help="batched report without the plain item-by-item comparison")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the 16-vehicle serving replay (FIFO vs continuous batching)")
    ap.add_argument("--serving-seconds", type=float, default=60.0,
                    help="length of the serving schedule (nominal-rate replay)")
    ap.add_argument("--no-grids", action="store_true",
                    help="skip the grid-A sweep and the grid-B infill protocol")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 256 MiB device-to-device copy (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 4}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the path would shard by spatial tile with an r-halo)", file=sys.stderr)
        sys.exit(2)

    sched = None
    if not args.no_serving:
        sched = serving_schedule_for_bench(args.serving_seconds)

    import numpy as np
    import torch

    import paper_2505_22675_amd as ag
    from gen import GridSpec, checksum, workload_cfg2

    dev = torch.device("cuda:0")
    log("generating 2M-sounding swath workload")
    s = workload_cfg2()
    digest = checksum(s.x, s.y, s.z)
    x, y, z = (torch.from_numpy(a).to(dev) for a in (s.x, s.y, s.z))
    grid = ag.auv_grid_create(s.grid)
    up_desc = GridSpec(s.grid.x0, s.grid.y0, s.grid.dx / 2, s.grid.dy / 2,
                       2 * s.grid.nx, 2 * s.grid.ny)
    ws_bytes = ag.auv_bin_workspace_size(grid, s.n, s.radius, 0)
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)
    shape = (s.grid.ny, s.grid.nx)
    z_out = torch.empty(shape, dtype=torch.float32, device=dev)
    nn_idx = torch.empty(shape, dtype=torch.int32, device=dev)
    nn_z = torch.empty(shape, dtype=torch.float32, device=dev)
    up = torch.empty((up_desc.ny, up_desc.nx), dtype=torch.float32, device=dev)
    params = ag.idw_params(s.power, s.radius, s.min_pts, s.max_pts)
    stream = torch.cuda.current_stream()

    def step(ev=None):
        if ev is not None:
            ev[0].record(stream)
        bins = ag.auv_bin_points(grid, x, y, z, s.radius, 0, ws=ws, stream=stream)
        if ev is not None:
            ev[1].record(stream)
        ag.auv_interp_idw(grid, bins, params, z_out, None, nn_idx, nn_z, stream=stream)
        if ev is not None:
            ev[2].record(stream)
        ag.auv_resample_bilinear(z_out, s.grid, up, up_desc, stream=stream)
        if ev is not None:
            ev[3].record(stream)
        return bins

    log(f"warmup {args.warmup} steps")
    for _ in range(args.warmup):
        bins = step()
    torch.cuda.synchronize()

    K = args.steps
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(K)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(K):
        bins = step(evs[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / K
    stage = np.array([[evs[k][j].elapsed_time(evs[k][j + 1]) for j in range(3)]
                      for k in range(K)])
    st_ms = stage.mean(axis=0)
    step_ev = np.array([evs[k][0].elapsed_time(evs[k][3]) for k in range(K)])
    log(f"timed {K} steps: {ms_per_step:.4f} ms/step; stages bin/idw/bilinear = "
        f"{st_ms[0]:.4f}/{st_ms[1]:.4f}/{st_ms[2]:.4f} ms")
    nan_frac = float(torch.isnan(z_out).float().mean().item())

    nodes = s.grid.nx * s.grid.ny
    _, _, counts = ag.auv_bins_export(bins)
    n_binned = counts[0]
    # algorithmic bytes per launch of each single-kernel stage
    alg = {
        "idw": n_binned * 20 + nodes * 12,          # binned SoA in, z + nn idx + nn z out
        "bilinear": nodes * 4 + up_desc.nx * up_desc.ny * 4,
    }
    dur = {"idw": st_ms[1], "bilinear": st_ms[2]}
    dom = max(dur, key=dur.get)
    achieved = alg[dom] / (dur[dom] * 1e-3) / 1e9
    kernel_names = {"idw": "k_idw_window", "bilinear": "k_bilinear"}
    roofline = {"bound": "hbm", "kernel": kernel_names[dom], "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": None, "algorithmic_bytes": int(alg[dom]),
                "avg_launch_ms": round(float(dur[dom]), 5)}

    roofline["traffic"] = traffic_from_profile(kernel_names[dom])
    roofline["traffic_source"] = (profile_source("hbm_traffic_swath2M.md", kernel_names[dom])
                                  if roofline["traffic"] is not None else None)
    # the algorithmic ALU fraction: in-radius pairs (every selected member of
    # every node, counted by one extra IDW launch with counts) times the ops a
    # pair needs, over the launch time, against the chip's lane-op rate
    if dom == "idw":
        cnt = torch.empty(shape, dtype=torch.int32, device=dev)
        ag.auv_interp_idw(grid, bins, params, z_out, cnt, nn_idx, nn_z, stream=stream)
        torch.cuda.synchronize()
        pairs = int(cnt.sum(dtype=torch.int64).item())
        del cnt
        alu_ops = pairs * ALU_OPS_PER_PAIR / (dur[dom] * 1e-3)
        roofline["alu"] = {"pairs": pairs, "ops_per_pair": ALU_OPS_PER_PAIR,
                           "achieved_lane_ops_per_s": round(alu_ops, 1),
                           "peak_lane_ops_per_s": LANE_OPS_PEAK,
                           "frac": round(alu_ops / LANE_OPS_PEAK, 4)}
        rel = max(("hbm", roofline["frac"]), ("alu", roofline["alu"]["frac"]),
                  key=lambda t: t[1])
        roofline["relevant"] = {"bound": rel[0], "frac": rel[1]}
    # issue rate: the profiled VALU instruction count (overhead included) over
    # the live launch time against the chip's issue rate
    valu = valu_from_profile(kernel_names[dom])
    roofline["valu_issue"] = None if valu is None else {
        "instructions": valu, "achieved_per_s": round(valu / (dur[dom] * 1e-3), 1),
        "peak_per_s": VALU_ISSUE_PEAK,
        "frac": round(valu / (dur[dom] * 1e-3) / VALU_ISSUE_PEAK, 4),
        "source": profile_source("valu_issue_swath2M.md", kernel_names[dom])}

    # the practical ceiling in this run: a 256 MiB device-to-device copy
    ca = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    cb = torch.empty_like(ca)
    copy_ms = _median_ms(lambda: cb.copy_(ca), stream, 20)
    roofline["copy_GBs"] = round(2 * ca.numel() * 4 / (copy_ms * 1e-3) / 1e9, 1)
    del ca, cb
    log(f"device copy: {roofline['copy_GBs']:.0f} GB/s")

    # cold steps: 512 MiB read before each one, so that no input or
    # intermediate of the previous step is left in the 256 MB last-level cache
    # (a read, not a write: dirty lines of a write flush would drain during
    # the step and slow its own writes)
    flush = torch.ones(128 << 20, dtype=torch.float32, device=dev)
    cold_ev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(20)]
    for k in range(20):
        flush.sum()
        step(cold_ev[k])
    torch.cuda.synchronize()
    del flush
    cold_stage = np.array([[cold_ev[k][j].elapsed_time(cold_ev[k][j + 1]) for j in range(3)]
                           for k in range(20)])
    cold_step = np.array([cold_ev[k][0].elapsed_time(cold_ev[k][3]) for k in range(20)])
    cold = {"steps": 20, "flush_read_bytes": 512 << 20,
            "step_ms_median": round(float(np.median(cold_step)), 5),
            "step_ms_min": round(float(cold_step.min()), 5),
            "stages_ms_median": {n: round(float(v), 5) for n, v in
                                 zip(("bin", "idw_nn", "bilinear"), np.median(cold_stage, axis=0))}}
    log(f"cold steps (512 MiB read before each): median {cold['step_ms_median']:.4f} ms, "
        f"stages {cold['stages_ms_median']}")

    # next row: Catmull-Rom 2x of the same grid (not part of the step)
    cub = torch.empty_like(up)
    for _ in range(3):
        ag.auv_resample_bicubic(z_out, s.grid, cub, up_desc, stream=stream)
    ce = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(20)]
    for e0, e1 in ce:
        e0.record(stream)
        ag.auv_resample_bicubic(z_out, s.grid, cub, up_desc, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    cub_ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ce]))
    cub_gbs = alg["bilinear"] / (cub_ms * 1e-3) / 1e9
    bicubic = {"workload": "Catmull-Rom 2x of the 4096^2 IDW grid to 8192^2, bilinear fallback "
                           "at NaN taps", "ms": round(cub_ms, 5), "achieved_GBs": round(cub_gbs, 1),
               "hbm_frac": round(cub_gbs / HBM_PEAK_GBS, 4),
               "nan_nodes": int(torch.isnan(cub).sum().item())}
    log(f"bicubic 2x: {cub_ms:.4f} ms ({cub_gbs:.0f} GB/s)")

    # next row: ordinary kriging 2x of the same grid, range three source cells
    krig = torch.empty_like(up)
    krig_range = 3.0 * s.grid.dx
    for _ in range(3):
        ag.auv_resample_kriging(z_out, s.grid, krig, up_desc, krig_range, stream=stream)
    ke = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(20)]
    for e0, e1 in ke:
        e0.record(stream)
        ag.auv_resample_kriging(z_out, s.grid, krig, up_desc, krig_range, stream=stream)
        e1.record(stream)
    torch.cuda.synchronize()
    krig_ms = float(np.median([e0.elapsed_time(e1) for e0, e1 in ke]))
    krig_gbs = alg["bilinear"] / (krig_ms * 1e-3) / 1e9
    kriging = {"workload": "ordinary kriging 2x of the 4096^2 IDW grid to 8192^2, 5x5 window, "
                           f"exponential variogram range {krig_range:g} m, bilinear fallback at "
                           "NaN windows", "ms": round(krig_ms, 5),
               "nodes_per_s": round(up.numel() / (krig_ms * 1e-3), 1),
               "achieved_GBs": round(krig_gbs, 1), "hbm_frac": round(krig_gbs / HBM_PEAK_GBS, 4),
               "nan_nodes": int(torch.isnan(krig).sum().item())}
    kv = valu_from_profile("k_kriging")
    kriging["valu_issue"] = None if kv is None else {
        "instructions": kv, "achieved_per_s": round(kv / (krig_ms * 1e-3), 1),
        "peak_per_s": VALU_ISSUE_PEAK, "frac": round(kv / (krig_ms * 1e-3) / VALU_ISSUE_PEAK, 4),
        "note": "counts exp/sqrt, which issue beside the main VALU: issue-bound, not a utilisation"}
    log(f"kriging 2x: {krig_ms:.4f} ms ({krig_gbs:.0f} GB/s)")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(s, up_desc, nodes)

    precision = None
    if not args.no_precision:
        precision = precision_report(ag, dev)

    batched = None
    if not args.no_batched:
        batched = batched_report(ag, dev, with_plain=not args.no_plain_batch,
                                 tune_in=args.batch_tune, tune_out=args.save_batch_tune)

    serving = None
    if not args.no_serving:
        serving = serving_report(ag, dev, sched, args.serving_seconds)
        del sched

    grid_a = grid_b = None
    if not args.no_grids:
        grid_a = grid_a_sweep(ag, dev, with_cpu=not args.no_cpu_baseline)
        grid_b = grid_b_report(ag, dev, with_cpu=not args.no_cpu_baseline)

    value = nodes / (ms_per_step * 1e-3)
    rec = {
        "metric": METRIC, "value": round(value, 1), "unit": "grid nodes/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "multibeam swath, 2M soundings (8 lines x 625 pings x 400 beams) "
                               "-> IDW p=2 r=6 m k=16 + nearest on 4096^2 @ 2 m, "
                               "bilinear 2x to 8192^2 @ 1 m",
                   "soundings": s.n, "grid": [s.grid.nx, s.grid.ny], "input_sha": digest,
                   "n_binned": int(n_binned)},
        "stages_ms": {"bin": round(float(st_ms[0]), 5), "idw_nn": round(float(st_ms[1]), 5),
                      "bilinear": round(float(st_ms[2]), 5)},
        "step_ms_events": {"median": round(float(np.median(step_ev)), 5),
                           "min": round(float(step_ev.min()), 5)},
        "cache": "timed steps run back to back: the step writes 268 MB of bilinear output, "
                 "more than the 256 MB last-level cache, but part of its inputs can stay "
                 "resident; `cold` repeats the step after a 512 MiB read",
        "cold": cold,
        "nan_frac": round(nan_frac, 4),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "precision_utm": precision,
        "bicubic": bicubic,
        "kriging": kriging,
        "batched_tiles": batched,
        "serving": serving,
        "grid_a_sweep": grid_a,
        "grid_b_infill": grid_b,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
