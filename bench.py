"""Throughput benchmark of the photon transport on one MI355X.

One step = one launch of the whole transport (on-device emission, BVH
closest-hit traversal, bulk absorption, Rayleigh scattering, surface and
Fresnel interactions, detection tally) over a batch of photons on the
DARWIN-scale synthetic TPC (about 4.75e5 triangles, 1,778 sensors), each
photon at its own uniform point of the active volume.  Inputs are resident in
HBM before the timed region.  Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--photons N]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "photons propagated/sec on DARWIN-scale TPC mesh; gradient-pass overhead vs forward"
HBM_PEAK = 8.0e12  # B/s, MI355X HBM3E
# VALU lane operations per second: 256 CUs x 4 SIMDs, each issuing one wave64
# instruction every 4 cycles (16 lanes per cycle), at 2.4 GHz; the same as the
# 78.6 TFLOP/s FP32 multiply-add figure counted in instructions instead of flops
VALU_LANE_PEAK = 256 * 4 * 16 * 2.4e9
# Algorithmic work per unit (what the method must compute; not what the kernel
# executes): VALU lane operations of one BVH4 node visit (four slab tests and
# the ordering of the hits), one watertight triangle test and the rest of a
# photon-step (free paths, interaction, random numbers), and the bytes a node
# visit and a triangle test fetch (a 128-B node, a 64-B triangle).
OPS_NODE, OPS_TRI, OPS_STEP = 64, 35, 150
NODE_BYTES, TRI_BYTES = 128, 64
# what decides the profiled launch: the built library (kernel code, BVH
# construction, launch defaults; the build is deterministic, and comments do
# not change it) and the Python defaults that choose the BVH options
PROFILED_FILES = ["paper_2203_14354_amd/libxephot.so", "paper_2203_14354_amd/runtime.py"]
PROFILES = os.path.join(ROOT, "profiles")
TRAFFIC_FILE = os.path.join(PROFILES, "darwin_tpc_hbm_traffic.md")
VALU_FILE = os.path.join(PROFILES, "propagate_darwin_tpc_valu_counters.md")
L2_FILE = os.path.join(PROFILES, "propagate_darwin_tpc_l2_requests.md")
STREAM_FILE = os.path.join(PROFILES, "stream_read_bandwidth_probe.md")


def kernel_hash() -> str:
    h = hashlib.sha256()
    for p in PROFILED_FILES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_values(path: str, photons_per_launch=None):
    """`key: number` lines of a committed rocprofv3 summary.  With
    photons_per_launch given, None unless the summary was taken on the current
    library at that launch size."""
    if not os.path.exists(path):
        return None
    vals = {}
    for m in re.finditer(r"^([A-Za-z0-9_]+):\s*([0-9a-f.eE+-]+)\s*$", open(path).read(), re.M):
        vals[m.group(1)] = m.group(2)
    if photons_per_launch is not None:
        if vals.get("library_sha256_16") != kernel_hash():
            return None
        if int(float(vals.get("photons_per_launch", -1))) != photons_per_launch:
            return None
    out = {}
    for k, v in vals.items():
        try:
            out[k] = float(v)
        except ValueError:
            pass
    return out


def timed_launches(fn, n, torch):
    """Run fn() n times; per-launch HIP event durations (s) and wall time (s)."""
    evs = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        evs.append((a, b))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return [a.elapsed_time(b) * 1e-3 for a, b in evs], wall


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--photons", type=int, default=100_000_000)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the gradient-overhead, batched, map, timing and spectrum measurements")
    ap.add_argument("--cache-probe", action="store_true",
                    help="only measure streaming-read bandwidth from buffers resident in the L2 "
                         "caches (16 MB), the Infinity Cache (64-192 MB) and HBM (8 GB)")
    ap.add_argument("--valu-probe", action="store_true",
                    help="only measure the VALU issue rate of kernels of known instruction count "
                         "(FP32 multiply-add, FP32 reciprocal, integer xor-add)")
    ap.add_argument("--calibration-copy", type=int, default=0, metavar="BYTES",
                    help="also run one device-to-device copy of BYTES bytes (a known-traffic "
                         "kernel for scaling rocprofv3 FETCH_SIZE / WRITE_SIZE)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the transport library runs on one GPU", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2203_14354_amd import workloads as W
    from paper_2203_14354_amd.runtime import Detector

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    if args.cache_probe:
        print(json.dumps(cache_probe(torch, dev)), flush=True)
        return
    if args.valu_probe:
        print(json.dumps(valu_probe(torch, dev)), flush=True)
        return
    if args.calibration_copy > 0:
        a = torch.ones(args.calibration_copy // 4, dtype=torch.float32, device=dev)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    mesh = W.darwin()
    det = Detector(mesh, device=0)
    wl = W.darwin_tpc(n_photons=args.photons, seed=args.seed, mesh=mesh)
    ds = det.sources(wl.sources)
    hit_map = torch.zeros((1, det.n_channels), dtype=torch.int32, device=dev)
    N = wl.sources.n_photons
    step_no = [0]

    def step():
        hit_map.zero_()
        det.propagate(ds, seed=args.seed, pid_base=step_no[0] * N, hit_map=hit_map)
        step_no[0] += 1

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    durations, wall = timed_launches(step, args.steps, torch)
    ms_per_step = wall / args.steps * 1e3
    value = N * args.steps / wall

    # counting launch (untimed): nodes visited, triangles tested, steps, flags
    cnt = det.propagate(ds, seed=args.seed, pid_base=0, stats=True)
    torch.cuda.synchronize()
    st = cnt["stats"].cpu().tolist()
    kern_s = statistics.mean(durations)
    roofline = roofline_of(st, kern_s, N)
    extras = {}
    if not args.no_extras:
        extras.update(gradient_overhead(torch, W, Detector, dev))
        extras.update(gradient_overhead_darwin(torch, W, det, mesh, dev))
        extras.update(batched_vs_plain(torch, W, Detector, dev))
        extras.update(lce_map_rate(torch, W, dev))
        extras.update(arrival_time_and_losses(torch, W, Detector, mesh, det, dev, args.photons))
        extras.update(spectrum_cost(torch, W, det, mesh, dev))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(W, mesh, args.seed)

    line = {
        "metric": METRIC, "value": value, "unit": "photons/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": "darwin_tpc", "photons_per_step": N,
                   "triangles": int(mesh.n_triangles), "sensors": int(mesh.n_sensors),
                   "source": "uniform in r<=1.299 m, -2.597<=z<=-0.001 m, isotropic, 175 nm",
                   "bvh_nodes": det.bvh["n_nodes"], "bvh_references": det.bvh["n_references"],
                   "bvh_depth": det.bvh["depth"],
                   "bvh_max_stack": det.bvh["max_stack"]},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "per_launch": {"steps_per_photon": st[9] / N, "photon_steps_per_s": value * st[9] / N,
                       "nodes_per_step": st[10] / st[9],
                       "triangles_per_step": st[11] / st[9],
                       "search_lane_utilization": (st[13] / st[12]) if st[12] else None,
                       "detected_fraction": st[1] / N, "bulk_absorbed_fraction": st[4] / N,
                       "surface_absorbed_fraction": st[3] / N,
                       "phase_cycle_fraction": st[16] / max(st[16] + st[17], 1),
                       "lane_steps_per_phase": st[9] / max(st[15], 1),
                       "geometry_errors": st[8], "escaped": st[5], "max_steps": st[6],
                       "nan_aborts": st[7]},
        "library_sha256_16": kernel_hash(),
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


def roofline_of(st, kern_s, n_photons):
    """Roofline of the transport kernel for one launch of n_photons photons
    whose average duration kern_s was measured with HIP events on its stream.

    The binding resource is VALU issue: the calibrated shader-sequencer
    counters (committed summary) show a VALU instruction issuing in about 89 %
    of the SIMD cycles, while the requests reaching L2 and the bytes leaving
    it are about a fifth and a quarter of the streaming rates measured for
    those levels.  `achieved` is the launch's algorithmic VALU work (per node
    visit, triangle test and photon-step, times the counts of the counting
    launch) per second against the VALU lane-operation peak; the executed
    work, the lane activity and the memory levels come from the summaries
    when they were taken on the current library."""
    n_steps, n_nodes, n_tris = st[9], st[10], st[11]
    ops = OPS_NODE * n_nodes + OPS_TRI * n_tris + OPS_STEP * n_steps
    achieved = ops / kern_s
    r = {"bound": "alu", "achieved": achieved / 1e12, "peak": VALU_LANE_PEAK / 1e12,
         "unit": "Tops/s", "frac": achieved / VALU_LANE_PEAK, "traffic": None,
         "kernel": "propagate_kernel<forward>", "avg_launch_s": kern_s,
         "algorithmic_lane_ops_per_launch": ops,
         "lane_ops_per_unit": {"node_visit": OPS_NODE, "triangle_test": OPS_TRI,
                               "photon_step": OPS_STEP}}
    tr = profile_values(TRAFFIC_FILE, n_photons)
    if tr:
        r["traffic"] = tr["hbm_bytes_per_launch"] / kern_s / 1e9
        r["traffic_unit"] = "GB/s"
        r["traffic_bytes_per_launch"] = tr["hbm_bytes_per_launch"]
    alg_bytes = NODE_BYTES * n_nodes + TRI_BYTES * n_tris
    r["hbm_algorithmic"] = {
        "achieved": alg_bytes / kern_s / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
        "frac": alg_bytes / kern_s / HBM_PEAK, "bytes_per_launch": alg_bytes,
        "note": "128 B per node visit + 64 B per triangle test; above 1 because the 100 MB of "
                "nodes and triangle records are read from L2 and the Infinity Cache, not HBM"}
    v = profile_values(VALU_FILE, n_photons)
    if v:
        r["valu"] = {"issue_busy": v["valu_issue_busy"],
                     "dual_issue_fraction": v["valu_dual_issue_fraction"],
                     "active_lane_fraction": v["valu_active_lane_fraction"],
                     "executed_lane_ops_per_photon_step": v["executed_lane_ops_per_photon_step"],
                     "executed_over_algorithmic": v["executed_lane_ops_per_launch"] / ops}
    l2, sp = profile_values(L2_FILE, n_photons), profile_values(STREAM_FILE)
    if l2 and sp:
        a2 = l2["l2_request_bytes_per_launch"] / kern_s / 1e9
        a3 = l2["past_l2_read_bytes_per_launch"] / kern_s / 1e9
        r["l2"] = {"achieved": a2, "peak": sp["l2_stream_read_GBps"], "unit": "GB/s",
                   "frac": a2 / sp["l2_stream_read_GBps"], "peak_kind": "measured streaming read"}
        r["past_l2"] = {"achieved": a3, "peak": sp["infinity_cache_stream_read_GBps"], "unit": "GB/s",
                        "frac": a3 / sp["infinity_cache_stream_read_GBps"],
                        "peak_kind": "measured streaming read from the Infinity Cache"}
    return r


def gradient_overhead(torch, W, Detector, dev):
    """Differentiable workload (small TPC + transparent plane, 1e7 photons):
    forward with fused FP64 gradient tallies, and the backward replay, each
    against plain forward transport on the same GPU."""
    wl = W.differentiable(photons_per_point=1_000_000)
    det = Detector(wl.mesh, device=0)
    ds = det.sources(wl.sources)
    hm = torch.zeros((1, det.n_channels), dtype=torch.int32, device=dev)
    g = torch.zeros((1, det.n_channels, 4), dtype=torch.float64, device=dev)
    gh = torch.ones((1, det.n_channels), dtype=torch.float32, device=dev)
    gp = torch.zeros(4, dtype=torch.float64, device=dev)
    runs = {
        "forward": lambda: det.propagate(ds, seed=1, hit_map=hm),
        "forward_fused_tallies": lambda: det.propagate(ds, seed=1, hit_map=hm, grad=g),
        "backward_replay": lambda: det.backward(ds, gh, seed=1, grad_params=gp),
    }
    t = {}
    for k, fn in runs.items():
        fn()
        d, _ = timed_launches(fn, 5, torch)
        t[k] = statistics.median(d)
    n = wl.sources.n_photons
    return {"gradient_overhead": {
        "workload": "differentiable: small TPC + transparent plane, 1e7 photons",
        "forward_photons_per_s": n / t["forward"],
        "fused_tallies_over_forward": t["forward_fused_tallies"] / t["forward"],
        "forward_plus_backward_over_forward": (t["forward"] + t["backward_replay"]) / t["forward"],
        "backward_replay_over_forward": t["backward_replay"] / t["forward"]}}


def gradient_overhead_darwin(torch, W, det, mesh, dev, n=20_000_000):
    """The same ratios on the DARWIN-scale workload (2e7 photons; gradients
    with respect to the LXe lengths, 1,778 channels x 4 FP64 scores)."""
    ds = det.sources(W.darwin_tpc(n_photons=n, mesh=mesh).sources)
    hm = torch.zeros((1, det.n_channels), dtype=torch.int32, device=dev)
    g = torch.zeros((1, det.n_channels, 4), dtype=torch.float64, device=dev)
    gh = torch.ones((1, det.n_channels), dtype=torch.float32, device=dev)
    gp = torch.zeros(4, dtype=torch.float64, device=dev)
    runs = {
        "forward": lambda: det.propagate(ds, seed=2, hit_map=hm),
        "forward_fused_tallies": lambda: det.propagate(ds, seed=2, hit_map=hm, grad=g),
        "backward_replay": lambda: det.backward(ds, gh, seed=2, grad_params=gp),
    }
    t = {}
    for k, fn in runs.items():
        fn()
        d, _ = timed_launches(fn, 3, torch)
        t[k] = statistics.median(d)
    return {"gradient_overhead_darwin": {
        "workload": f"darwin_tpc, {n} photons, gradients for the LXe absorption and Rayleigh lengths",
        "forward_photons_per_s": n / t["forward"],
        "fused_tallies_over_forward": t["forward_fused_tallies"] / t["forward"],
        "forward_plus_backward_over_forward": (t["forward"] + t["backward_replay"]) / t["forward"],
        "backward_replay_over_forward": t["backward_replay"] / t["forward"]}}


def batched_vs_plain(torch, W, Detector, dev):
    """4096 log-normal S1 sources in one persistent launch vs plain forward of
    the same photon count from one source list without per-event maps."""
    wl = W.batched_s1()
    det = Detector(wl.mesh, device=0)
    ds = det.sources(wl.sources)
    n = wl.sources.n_photons
    hm = torch.zeros((wl.sources.n_events, det.n_channels), dtype=torch.int32, device=dev)
    plain_src = W.point_sources(wl.sources.positions, counts=None,
                                count_per_source=int(-(-n // len(wl.sources.positions))))
    dp = det.sources(plain_src)
    hm1 = torch.zeros((1, det.n_channels), dtype=torch.int32, device=dev)
    fb = lambda: det.propagate(ds, seed=2, hit_map=hm)
    fp = lambda: det.propagate(dp, seed=2, hit_map=hm1, n_photons=n)
    fb()
    fp()
    db, _ = timed_launches(fb, 5, torch)
    dpl, _ = timed_launches(fp, 5, torch)
    # the same launch autotuned and replayed from a captured HIP graph (the map
    # is cleared by a fill kernel inside the graph)
    from paper_2203_14354_amd.batched import BatchedRunner
    runner = BatchedRunner(det, wl.sources, seed=2, autotune=True, use_graph=True)
    runner.run()
    dg, _ = timed_launches(runner.run, 5, torch)
    return {"batched_s1": {"workload": f"4096 log-normal sources, {n} photons, per-event maps",
                           "photons_per_s": n / statistics.median(db),
                           "graph_autotuned_photons_per_s": n / statistics.median(dg),
                           "autotuned_launch": runner.launch,
                           "plain_forward_photons_per_s": n / statistics.median(dpl)}}


def lce_map_rate(torch, W, dev):
    """64^3 equal-volume cells x 1e4 photons (2.6e9 photons) on the small TPC
    with the transparent plane: {top, bottom} counts and FP64 gradients per cell."""
    from paper_2203_14354_amd import lcemap
    det = lcemap.tpc1_lce_map_detector()
    cen = W.equal_volume_cell_centroids(64, 64, 64, W.TPC1_SRC_R, -W.TPC1_SRC_ZHALF,
                                        W.TPC1_SRC_ZHALF)
    lcemap.lce_map(det, cen[:16384], 100, seed=4)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hits, g = lcemap.lce_map(det, cen, 10_000, seed=4, batch_cells=16384)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    n = len(cen) * 10_000
    lce = hits.sum(dim=1).double() / 10_000
    return {"lce_map": {"workload": "small TPC + plane, 64^3 cells x 1e4 photons, "
                                    "{top, bottom} + 4 FP64 gradients per cell",
                        "photons": n, "seconds": dt, "photons_per_s": n / dt,
                        "mean_lce": float(lce.mean()), "min_lce": float(lce.min()),
                        "max_lce": float(lce.max())}}


def arrival_time_and_losses(torch, W, Detector, mesh, det, dev, n_photons):
    """DARWIN-scale workload with the NR scintillation profile: forward with
    the per-event arrival-time histogram (1 ns bins) and the loss table against
    plain forward; t90 of all detected photons; the average of per-position
    t90 over 64 point sources; the loss table folded into the paper's
    components."""
    from paper_2203_14354_amd import runtime
    groups, names = W.loss_components(mesh)
    det.set_loss_groups(groups, len(names))
    src = W.with_scintillation(W.darwin_tpc(n_photons=n_photons, mesh=mesh).sources)
    ds = det.sources(src)
    n = src.n_photons
    hm = torch.zeros((1, det.n_channels), dtype=torch.int32, device=dev)
    th = torch.zeros((1, 2048), dtype=torch.int32, device=dev)
    lt = torch.zeros((len(names) + len(det.materials), 8), dtype=torch.int64, device=dev)
    plain = lambda: det.propagate(ds, seed=5, hit_map=hm)
    tallied = lambda: det.propagate(ds, seed=5, hit_map=hm, time_hist=th, time_bin_ns=1.0, loss=lt)
    plain()
    tallied()
    dp, _ = timed_launches(plain, 3, torch)
    dt_, _ = timed_launches(tallied, 3, torch)
    th.zero_()
    lt.zero_()
    tallied()
    t90_all = float(runtime.time_quantile(th, 1.0, 0.9)[0])
    loss = lt.cpu().numpy().astype(np.float64) / n
    ng = len(names)
    absorbed = {names[g]: float(loss[g, 2] + loss[g, 3]) for g in range(ng)}
    for m, mname in enumerate(W.DARWIN_MATERIAL_NAMES[:len(det.materials)]):
        absorbed[mname + " (bulk)"] = float(loss[ng + m, 4])
    # per-position t90: 64 points uniform in the active volume, 1e5 photons each
    pts = W.uniform_points_in_cylinder(64, W.DARWIN_SRC_R, W.DARWIN_SRC_ZLO, W.DARWIN_SRC_ZHI, seed=9)
    ps = W.with_scintillation(W.point_sources(pts, count_per_source=100_000, per_source_events=True))
    pth = det.propagate(ps, seed=6, time_hist=2048, time_bin_ns=1.0)["time_hist"]
    t90_pos = runtime.time_quantile(pth, 1.0, 0.9).cpu().numpy()
    return {"arrival_time_and_losses": {
        "workload": "darwin_tpc with the NR scintillation profile (3.5 / 24 ns, singlet 0.66), "
                    f"{n} photons; time histogram 2048 x 1 ns; loss table by component",
        "tallies_over_forward": statistics.median(dt_) / statistics.median(dp),
        "photons_per_s_with_tallies": n / statistics.median(dt_),
        "t90_all_detected_ns": t90_all,
        "t90_mean_over_64_positions_ns": float(np.nanmean(t90_pos)),
        "t90_min_max_over_positions_ns": [float(np.nanmin(t90_pos)), float(np.nanmax(t90_pos))],
        "detected_fraction": float(loss[:, 1].sum()),
        "absorbed_fraction_by_component": absorbed}}


def cache_probe(torch, dev):
    """Streaming-read bandwidth of buffers that fit the eight 4 MB L2 caches
    (16 MB: each XCD's workgroups touch one eighth), the 256 MB Infinity Cache
    (32 to 192 MB) and only HBM (8 GB): one launch reads each buffer
    repeatedly (about 16 GB per launch), every thread with four loads in
    flight (the grid shrinks for small buffers so that each thread has four
    vectors per pass); HIP events time 5 launches."""
    import ctypes
    from paper_2203_14354_amd import _lib
    lib = _lib.load()
    out = torch.empty(2048 * 256, dtype=torch.float32, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    rates = {}
    for name, mb in (("l2_16MB", 16), ("infinity_cache_32MB", 32), ("infinity_cache_64MB", 64),
                     ("infinity_cache_128MB", 128), ("infinity_cache_192MB", 192),
                     ("hbm_8GB", 8192)):
        x = torch.ones(mb * (1 << 20) // 4, dtype=torch.float32, device=dev)
        n_vec = x.numel() // 4
        blocks = int(max(256, min(2048, n_vec // (4 * 256))))
        passes = max(1, (16 << 30) // (mb << 20))
        run = lambda: _lib.check(lib.xp_stream_read(ctypes.c_void_p(x.data_ptr()), n_vec, passes,
                                                    blocks, ctypes.c_void_p(out.data_ptr()), stream))
        run()
        d, _ = timed_launches(run, 5, torch)
        rates[name] = n_vec * 16 * passes / statistics.median(d) / 1e9
        del x
    return {"stream_read_GBps": rates}


# VALU instructions one iteration of the probe loop issues per wave (64
# steps on eight chains, one to three instructions per step by kind)
VALU_PROBE_KINDS = {0: ("fp32_fma", 64), 1: ("fp32_rcp", 64), 2: ("int32_xor_add", 128),
                    3: ("fp32_fma_and_int32_xor_add", 192), 4: ("fp32_fma_and_rcp", 128),
                    5: ("u64_mad_and_move", 128)}


def valu_probe(torch, dev, iters=20_000):
    """VALU issue rate of kernels of known instruction count: eight workgroups
    of 256 threads per CU (eight waves per SIMD) run `iters` iterations of
    the probe loop; HIP events time 5 launches.  Reports wave-instructions per
    second and the SIMD cycles (at the 2.4 GHz peak clock) per wave64
    instruction."""
    import ctypes
    from paper_2203_14354_amd import _lib
    lib = _lib.load()
    n_cu = torch.cuda.get_device_properties(dev).multi_processor_count
    blocks = n_cu * 8
    out = torch.empty(blocks * 256, dtype=torch.float32, device=dev)
    stream = ctypes.c_void_p(torch.cuda.current_stream(dev).cuda_stream)
    res = {"compute_units": n_cu, "blocks": blocks, "iters": iters}
    for kind, (name, per_iter) in VALU_PROBE_KINDS.items():
        run = lambda: _lib.check(lib.xp_valu_probe(kind, iters, blocks,
                                                   ctypes.c_void_p(out.data_ptr()), stream))
        run()
        d, _ = timed_launches(run, 5, torch)
        t = statistics.median(d)
        instr = blocks * 4 * per_iter * iters  # wave-instructions (4 waves per block)
        res[name] = {"seconds": t, "wave_instructions": instr,
                     "wave_instructions_per_s": instr / t,
                     "cycles_per_instruction_per_simd": n_cu * 4 * t * 2.4e9 / instr}
    return {"valu_probe": res}


def spectrum_cost(torch, W, det, mesh, dev, n=20_000_000):
    """DARWIN-scale transport with per-photon wavelengths from the Gaussian
    spectrum (174.8 nm, FWHM 10.2 nm) against one line: the extra draw per
    photon; without dispersion tables the LCE does not change."""
    out = {}
    for name, src in (("one_line", W.darwin_tpc(n_photons=n, mesh=mesh).sources),
                      ("gaussian_spectrum", W.with_spectrum(W.darwin_tpc(n_photons=n, mesh=mesh).sources))):
        ds = det.sources(src)
        hm = torch.zeros((1, det.n_channels), dtype=torch.int32, device=dev)
        run = lambda: det.propagate(ds, seed=3, hit_map=hm)
        run()
        d, _ = timed_launches(run, 3, torch)
        hm.zero_()
        run()
        out[name] = {"photons_per_s": n / statistics.median(d), "lce": int(hm.sum()) / n}
    return {"spectrum": {"workload": f"darwin_tpc, {n} photons", **out,
                         "spectrum_over_one_line_time": out["one_line"]["photons_per_s"]
                         / out["gaussian_spectrum"]["photons_per_s"]}}


def cpu_baseline(W, mesh, seed, reps=3):
    """The FP64 oracle as it stands (OpenMP over photons on the host threads
    it is given, its own BVH for the closest hit), median of `reps` runs on
    each of: the small-TPC workload in full (1e5 photons); photon ids
    0 .. 1e6-1 of the DARWIN-scale workload (the GPU's first 1e6 photons);
    the differentiable workload in full (1e7 photons, FP64 gradient
    tallies).  `value` is the DARWIN-scale rate, the benchmark's workload."""
    import oracle
    threads = oracle.max_threads()

    def median_rate(scene, src, **kw):
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            oracle.run(scene, src, seed=seed, records=False, hit_map=True, **kw)
            ts.append(time.perf_counter() - t0)
        return src.n_photons / statistics.median(ts), ts

    runs = {}
    wl1 = W.small_tpc()
    runs["small_tpc"] = median_rate(oracle.Scene(wl1.mesh, use_bvh=True), wl1.sources)
    src2 = W.darwin_tpc(n_photons=1_000_000, seed=seed, mesh=mesh).sources
    runs["darwin_tpc_first_1e6"] = median_rate(oracle.Scene(mesh, use_bvh=True), src2)
    wl4 = W.differentiable(photons_per_point=1_000_000)
    runs["differentiable"] = median_rate(oracle.Scene(wl4.mesh, use_bvh=True), wl4.sources,
                                         grad=True)
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    value = runs["darwin_tpc_first_1e6"][0]
    return {"value": value, "unit": "photons/s", "cores": threads, "kind": "oracle",
            "sample": f"photon ids 0..999999 of the DARWIN-scale workload, FP64, OpenMP on "
                      f"{threads} threads, median of {reps} runs",
            "per_core": value / threads, "cpu_model": model, "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0)),
            "configs": {k: {"photons_per_s": r, "per_core": r / threads,
                            "seconds": [round(t, 3) for t in ts]}
                        for k, (r, ts) in runs.items()}}


if __name__ == "__main__":
    main()
