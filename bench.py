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
import json
import os
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


def kernel_source_digest() -> str:
    """Digest of the HIP sources, to tell whether a committed counter profile
    still describes the kernels being timed."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2505_22675_amd", "csrc")
    for fn in sorted(os.listdir(csrc)):
        if fn.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, fn), "rb") as f:
                h.update(fn.encode())
                h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary
    (FETCH_SIZE and WRITE_SIZE, each scaled by the copy-kernel calibration).
    None when there is no summary or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic_swath2M.md")
    if not os.path.exists(path):
        return None
    rec = {}
    digest = None
    with open(path) as f:
        for line in f:
            if line.startswith("source_digest:"):
                digest = line.split(":", 1)[1].strip()
            if line.startswith("traffic_bytes "):
                _, name, val = line.split()
                rec[name] = int(val)
    if digest != kernel_source_digest():
        return None
    return rec.get(kernel)


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
    oz, oc, _ = oracle.idw(og, s.x, s.y, s.z, s.radius, s.power, s.min_pts, s.max_pts,
                           bin_log2=19, nthreads=host_threads())
    grid = ag.auv_grid_create(s.grid)
    x, y, z = (torch.from_numpy(a).to(dev) for a in (s.x, s.y, s.z))
    bins = ag.auv_bin_points(grid, x, y, z, s.radius, 0)
    out = {}
    names = {ag.AUV_P_FP32_REBASE: "fp64_rebase_fp32", ag.AUV_P_FP16_OFFSETS: "fp16_offsets",
             ag.AUV_P_FP32_ABSOLUTE: "fp32_absolute"}
    for prec, name in names.items():
        res = ag.grid_idw(grid, bins, power=s.power, min_pts=s.min_pts, max_pts=s.max_pts,
                          with_counts=True, precision=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            ag.grid_idw(grid, bins, power=s.power, min_pts=s.min_pts, max_pts=s.max_pts,
                        with_counts=True, precision=prec)
        e1.record()
        torch.cuda.synchronize()
        gz = res["z"].cpu().numpy().astype(np.float64)
        both = ~np.isnan(gz) & ~np.isnan(oz)
        err = np.abs(gz[both] - oz[both])
        rel = err / np.abs(oz[both])
        out[name] = {"max_abs_m": float(err.max()), "rms_m": float(np.sqrt((err ** 2).mean())),
                     "max_rel": float(rel.max()),
                     "nan_mask_mismatch": int((np.isnan(gz) != np.isnan(oz)).sum()),
                     "count_mismatch": int((res["cnt"].cpu().numpy() != oc).sum()),
                     "idw_ms": round(e0.elapsed_time(e1) / 5, 4)}
        log(f"  {name}: {out[name]}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the UTM-scale precision-variant error report")
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
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported: "
              "this build runs on a single GPU (the path would shard by spatial tile "
              "with an r-halo)", file=sys.stderr)
        sys.exit(2)

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
    log(f"timed {K} steps: {ms_per_step:.4f} ms/step; stages bin/idw/bilinear = "
        f"{st_ms[0]:.4f}/{st_ms[1]:.4f}/{st_ms[2]:.4f} ms")

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

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(s, up_desc, nodes)

    precision = None
    if not args.no_precision:
        precision = precision_report(ag, dev)

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
        "roofline": roofline,
        "cpu_baseline": cpu,
        "precision_utm": precision,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
