"""Throughput of the transient NLOS forward operator on one MI355X.

One step = the whole hot path on one seeded scene already resident in HBM,
one nlos_simulate call: depth/albedo/mask -> patch records and their
summaries -> pair evaluation, LDS binning, guard re-binning, jitter and
write-out.  Default workload: confocal 64x64 scan points on a 2x2 m
wall, 256x256-pixel depth map with a blob mask (~32k active patches),
T = 1024 bins of 8 ps, jitter FWHM 50 ps.

Prints one JSON line: value = scan-point x patch pairs per second (Gpairs/s)
over the timed steps, plus the dominant kernel's roofline figures (measured
with HIP events on the launch stream) and the FP64 oracle timed on the host
cores.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gpairs/s (scan pt×patch) + % FP32 peak; p50/p99 latency, batched vs plain"
FLOPS_CONFOCAL = 29      # nominal flops per confocal pair (formula written without FMA)
FLOPS_NONCONFOCAL = 48   # per non-confocal (laser, detector, patch) triple
FP32_PEAK_TFLOPS = 157.3  # MI355X published FP32 vector peak
# the same peak without packed FP32 (256 CU x 4 SIMD x 16 lanes x 2 flops per
# FMA x 2.4 GHz): the ceiling of kernels built with packed FP32 disabled
FP32_FMA_CEILING_TFLOPS = 78.6

# HBM bytes per launch of the cfg2 pair kernel from rocprofv3 counters
# (FETCH_SIZE 4297.2 KiB x 2.0 + WRITE_SIZE 16393.8 KiB x 1.0; the factors are
# what the same counters read for a 256 MiB device copy, see
# profiles/k_forward_cfg2_hbm_counters.md), valid only for the kernel sources
# they were taken on (hash below); any other source reports null.
TRAFFIC_BYTES = (4297.2 * 2.0 + 16393.8 * 1.0) * 1024
TRAFFIC_SOURCES = ("paper_2506_03747_amd/csrc/nlos_forward.hip", "paper_2506_03747_amd/csrc/nlos_device.h",
                   "paper_2506_03747_amd/csrc/nlos_internal.h")
TRAFFIC_HASH = "db2b6686818997be"


def traffic_for_sources():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return TRAFFIC_BYTES if h.hexdigest()[:16] == TRAFFIC_HASH else None

WORKLOADS = {
    "cfg2": "confocal 64x64 scan on 2x2 m wall, 256x256 patch depth map in [0.4,1.2] m with blob mask, "
            "albedo U[0,1], T=1024 x 8 ps, FWHM 50 ps, no stand-off",
    "cfg1": "confocal 32x32 scan on 1x1 m wall, stand-off 1 m, 64x64 patches at 0.5 m +/- 5 cm with blob "
            "mask, T=512 x 16 ps, FWHM 70 ps",
    "cfg3": "non-confocal 8x8 lasers x 128x128 detectors on 2x2 m wall, stand-off 2 m, 128x128 patches from "
            "two overlapping surfaces, T=2048 x 4 ps, FWHM 30 ps",
    "cfg5": "confocal 128x128 scan on 2x2 m wall, 128x128 patches (no mask), T=1024 x 8 ps, FWHM 50 ps",
}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="cfg2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests of the serving mix for the batched-vs-plain latency leg (0: skip)")
    ap.add_argument("--no-graph", action="store_true", help="skip the graph-replayed step timing")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the smooth forward / adjoint leg")
    ap.add_argument("--no-lct", action="store_true", help="skip the FFT-route leg")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MiB",
                    help="also run a plain device copy of this size (3 times), the known-size reference for "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the library runs the operator on a single MI355X "
              f"(--gpus {args.gpus} is not supported; sharding over several GPUs is described, not built)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2506_03747_amd as nl
    import scenes

    sc = scenes.by_name(args.workload)
    dev = "cuda"
    depth = torch.from_numpy(sc.depth).to(dev)
    albedo = torch.from_numpy(sc.albedo).to(dev) if sc.albedo is not None else None
    mask = torch.from_numpy(sc.mask).to(dev) if sc.mask is not None else None
    prm = nl.params_of(sc)
    npx = sc.n_patch_total
    patches = torch.empty((npx, 8), dtype=torch.float32, device=dev)
    n_act = torch.empty(1, dtype=torch.int32, device=dev)
    out = torch.empty(nl.out_shape(prm), dtype=torch.float32, device=dev)
    stream = torch.cuda.current_stream()

    import ctypes as C
    from paper_2506_03747_amd._native import Probe, check, lib
    need = C.c_size_t(0)
    check(lib().nlos_simulate_workspace_bytes(C.byref(prm), C.byref(nl.make_grid(sc.patch_grid)), C.byref(need)),
          "nlos_simulate_workspace_bytes")
    sim_ws = torch.empty(need.value, dtype=torch.uint8, device=dev)

    # the C-ABI arguments of the step, marshalled once (every buffer is fixed)
    grid_c = nl.make_grid(sc.patch_grid)
    ptr = lambda t: None if t is None else C.c_void_p(t.data_ptr())
    sim = lib().nlos_simulate
    pre = (C.byref(prm), C.byref(grid_c), ptr(depth), ptr(albedo), ptr(mask), ptr(patches), ptr(n_act), ptr(out),
           ptr(sim_ws), sim_ws.numel())
    evaluated = torch.zeros(1, dtype=torch.int64, device=dev)

    def step(ev=None, count=False):
        cur = torch.cuda.current_stream()
        probe = None
        if ev is not None or count:
            if ev is not None:
                # recorded here so torch knows the event; the library records it
                # again right before the pair kernel, which moves its timestamp there
                ev[0].record(cur)
            probe = C.byref(Probe(None if ev is None else ev[0].cuda_event,
                                  evaluated.data_ptr() if count else None))
        rc = sim(*pre, probe, C.c_void_p(cur.cuda_stream))
        if rc != 0:
            check(rc, "nlos_simulate")
        if ev is not None:
            ev[1].record(cur)

    if args.copy_calibration > 0:
        n_b = args.copy_calibration << 20
        src = torch.ones(n_b // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    P_act = int(n_act.item())
    H = nl.n_histograms(prm)
    pairs = H * P_act
    # pairs the pair kernel evaluates per launch (the rest are culled as
    # arriving past the window; the count does not depend on the schedule)
    evaluated.zero_()
    step(count=True)
    torch.cuda.synchronize()
    pairs_evaluated = int(evaluated.item())

    # timed region 1 (throughput): K steps back to back, bracketed only
    # (an event recorded between kernels costs several microseconds)
    t_ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    t_ev[0].record(stream)
    for i in range(args.steps):
        step()
    t_ev[1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = max(wall * 1e3, t_ev[0].elapsed_time(t_ev[1])) / args.steps

    # timed region 2 (kernel and step latency): the same K steps, each with
    # HIP events on the launch stream: before the pair kernel (recorded by the
    # library), after it, and between steps
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    step_ev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]
    torch.cuda.synchronize()
    step_ev[0].record(stream)
    for i in range(args.steps):
        step(evs[i])
        step_ev[i + 1].record(stream)
    torch.cuda.synchronize()

    graph = None
    if not args.no_graph:
        graph = [graph_leg(step, stream, args.steps, pairs, k) for k in (1, 10)]
    noise = noise_leg(out)

    kern_ms = np.array([a.elapsed_time(b) for a, b in evs])
    step_ms = np.array([step_ev[i].elapsed_time(step_ev[i + 1]) for i in range(args.steps)])
    value = pairs / (ms_per_step * 1e-3) / 1e9
    F = FLOPS_CONFOCAL if sc.laser is None else FLOPS_NONCONFOCAL
    kern_avg = float(kern_ms.mean())
    # algorithmic flops: F per evaluated pair (culled pairs cost no pair work)
    achieved = F * pairs_evaluated / (kern_avg * 1e-3) / 1e12
    achieved_all = F * pairs / (kern_avg * 1e-3) / 1e12

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        olib = oracle.load()
        sample = sc
        sub = None
        if sc.laser is not None:
            sub = np.sort(np.random.default_rng(0).choice(H, 512, replace=False)).astype(np.int32)
        times = []
        for _ in range(3):
            t = time.perf_counter()
            rec = oracle.patches(sample, lib=olib)
            oracle.forward(sample, rec, subset=sub, lib=olib)
            times.append(time.perf_counter() - t)
        n_h = H if sub is None else len(sub)
        cpu_pairs = n_h * P_act
        cpu = {"value": cpu_pairs / float(np.median(times)) / 1e9, "unit": "Gpairs/s",
               "cores": oracle.num_threads(olib), "kind": "oracle",
               "sample": (f"full {args.workload} step ({n_h} histograms x {P_act} patches, jitter "
                          f"included), fp64 brute force, median of 3 runs" if sub is None else
                          f"{n_h} of {H} histograms x {P_act} patches, median of 3 runs")}

    line = {
        "metric": METRIC, "value": round(value, 3), "unit": "Gpairs/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "histograms": H,
                   "patches_active": P_act, "patches_total": npx, "n_bins": sc.n_bins,
                   "pairs_per_step": pairs},
        # F x all pairs / kernel time (the throughput figure's flop rate) and
        # F x evaluated pairs / kernel time (the work the kernel really did)
        "pct_fp32_peak": round(100 * achieved_all / FP32_PEAK_TFLOPS, 2),
        "pct_fp32_peak_evaluated": round(100 * achieved / FP32_PEAK_TFLOPS, 2),
        "latency_ms": {"p50": round(float(np.percentile(step_ms, 50)), 5),
                       "p99": round(float(np.percentile(step_ms, 99)), 5)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 3), "peak": FP32_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(achieved / FP32_PEAK_TFLOPS, 4),
                     "traffic": traffic_for_sources() if args.workload == "cfg2" else None, "kernel": "k_forward",
                     "kernel_ms": round(kern_avg, 5), "flops_per_pair": F,
                     "pairs_evaluated": pairs_evaluated, "pairs_all": pairs,
                     "frac_all_pairs": round(achieved_all / FP32_PEAK_TFLOPS, 4),
                     "frac_of_unpacked_ceiling": round(achieved / FP32_FMA_CEILING_TFLOPS, 4)},
        "cpu_baseline": cpu,
        "graph": graph,
        "noise": noise,
        "serving": serving_leg(args.serving_requests) if args.serving_requests > 0 else None,
        "adjoint": None if args.no_adjoint else adjoint_leg(),
        "lct": None if args.no_lct else lct_leg(),
    }
    print(json.dumps(line), flush=True)


def noise_leg(tau, reps=20):
    """Poisson noise of the step's output frame (Algorithm 1 step 2.4 after
    the blur): frame variance -> sigma_n (nr = 2 dB) -> noisy frame."""
    import torch
    import paper_2506_03747_amd as nl
    noisy = torch.empty_like(tau)
    nl.add_poisson_noise(tau, 2.0, 1, out=noisy)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(reps):
        nl.add_poisson_noise(tau, 2.0, i, out=noisy)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    return {"elements": tau.numel(), "ms": round(ms, 4), "gelem_s": round(tau.numel() / (ms * 1e-3) / 1e9, 3)}


def graph_leg(step, stream, steps, pairs, per_replay=1):
    """The same step captured in a HIP graph (per_replay steps back to back
    in one graph) and replayed."""
    import torch
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        step()                      # warm-up on the capture stream
        torch.cuda.synchronize()
        with torch.cuda.graph(g, stream=side):
            for _ in range(per_replay):
                step()
    torch.cuda.synchronize()
    for _ in range(5):
        g.replay()
    torch.cuda.synchronize()
    reps = max(1, steps // per_replay)
    t0 = time.perf_counter()
    for _ in range(reps):
        g.replay()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / (reps * per_replay)
    return {"steps_per_replay": per_replay, "ms_per_step": round(ms, 5),
            "gpairs_s": round(pairs / (ms * 1e-3) / 1e9, 3)}


def adjoint_leg(reps=10):
    """Differentiable path on the 128x128 scan x 128x128 patch workload
    (T=1024 x 8 ps, FWHM 50 ps, smooth support ceil(6 sigma) = 16 bins):
    smooth forward, record adjoint and map adjoint, HIP-event timed."""
    import torch
    import scenes
    import paper_2506_03747_amd as nl
    sc = scenes.cfg5()
    d = torch.from_numpy(sc.depth).cuda()
    a = torch.from_numpy(sc.albedo).cuda()
    prm = nl.params_of(sc)
    rec, n = nl.patches_from_depth(d, sc.patch_grid, a, None)
    tau = nl.forward_smooth(prm, rec, n)
    G = torch.randn(tau.shape, generator=torch.Generator(device="cuda").manual_seed(5), device="cuda")
    gr = nl.adjoint(prm, rec, n, G)
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    pairs = sc.n_scan * int(n.item())
    t_s = timed(lambda: nl.forward_smooth(prm, rec, n, out=tau))
    t_a = timed(lambda: nl.adjoint(prm, rec, n, G, out=gr))
    t_m = timed(lambda: nl.patches_adjoint(sc.patch_grid, d, a, rec, n, gr))
    return {"workload": "cfg5: confocal 128x128 scan, 128x128 patches (no mask), T=1024 x 8 ps, FWHM 50 ps",
            "pairs": pairs, "smooth_ms": round(t_s, 4), "adjoint_ms": round(t_a, 4), "maps_ms": round(t_m, 4),
            "smooth_gpairs_s": round(pairs / (t_s * 1e-3) / 1e9, 3),
            "adjoint_gpairs_s": round(pairs / (t_a * 1e-3) / 1e9, 3)}


def lct_leg(reps=5):
    """The paper's FFT (light-cone) route beside the direct operator on the
    128x128 scan x 128x128 depth map workload without cosines (Eq. (1) as
    printed), T=1024 x 8 ps: time of each and their correlation."""
    import ctypes as C
    import torch
    import scenes
    import paper_2506_03747_amd as nl
    from paper_2506_03747_amd._native import check, lib
    sc = scenes.cfg5()
    sc.cosines = False
    d = torch.from_numpy(sc.depth).cuda()
    a = torch.from_numpy(sc.albedo).cuda()
    prm = nl.params_of(sc)
    out = nl.lct_forward(prm, d, a)
    rec, n = nl.patches_from_depth(d, sc.patch_grid, a, None, cosines=False)
    direct = nl.forward(prm, rec, n)
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    nb = C.c_size_t(0)
    check(lib().nlos_lct_workspace_bytes(C.byref(prm), C.byref(nb)), "nlos_lct_workspace_bytes")
    big = torch.empty(nb.value, dtype=torch.uint8, device="cuda")
    t_lct = timed(lambda: nl.lct_forward(prm, d, a, out=out, workspace=big))
    t_dir = timed(lambda: nl.forward(prm, rec, n, out=direct))
    corr = float(torch.corrcoef(torch.stack([out.flatten().double(), direct.flatten().double()]))[0, 1])
    return {"workload": "cfg5 without cosines: confocal 128x128 scan co-registered with the 128x128 depth map, "
                        "T=1024 x 8 ps, FWHM 50 ps", "lct_ms": round(t_lct, 3), "direct_ms": round(t_dir, 4),
            "corr_with_direct": round(corr, 4), "workspace_bytes": nb.value}


def serving_leg(n_req):
    """Batched vs plain serving of the uneven request mix: requests 0..n-1 of
    the serving mix (confocal, scan 32..128 squared, 4k..262k patches, T of
    512/1024/2048), Poisson arrivals at 1.5x the measured plain capacity, 2 GiB
    HBM budget (tick workspaces and requests in flight).  Batched: each tick
    is one graph launch on one of three overlapping streams; plain: one
    request at a time through the one-call path on one stream.  Latency =
    tick completion on the GPU minus arrival."""
    import torch
    import scenes
    from paper_2506_03747_amd import n_histograms, params_of, serving

    reqs = [scenes.cfg4_request(i) for i in range(n_req)]
    pairs = 0
    for r in reqs:
        present = (r.mask != 0) & (r.albedo > 0) & np.isfinite(r.depth) & (r.depth > 0)
        pairs += n_histograms(params_of(r)) * int(present.sum())
    staged = [serving.Server.stage(r) for r in reqs]
    budget = 2 << 30
    out = {"workload": f"serving mix: requests 0..{n_req - 1} (seed 4+i), confocal, scan U{{32..128}}^2, "
                       f"U[4k,262k] patches, T in {{512,1024,2048}}, 4-16 ps bins, 30-70 ps FWHM",
           "requests": n_req, "pairs": pairs, "hbm_budget_bytes": budget}
    # warm-up of both paths, then the plain capacity with every request waiting
    for mode in ("plain", "batched"):
        serving.Server(budget, mode=mode).serve(reqs[:8], np.zeros(8), staged=staged[:8])
    sat = serving.Server(budget, mode="plain").serve(reqs, np.zeros(n_req), staged=staged)
    cap = n_req / (sat.makespan_ms * 1e-3)
    rate = 1.5 * cap
    out["plain_capacity_req_s"] = round(cap, 2)
    out["arrival_rate_req_s"] = round(rate, 2)
    arrivals = serving.poisson_arrivals(n_req, rate, seed=4)
    for mode in ("plain", "batched"):
        res = serving.Server(budget, mode=mode).serve(reqs, arrivals, staged=staged)
        out[mode] = {"p50_ms": round(res.percentile(50), 3), "p99_ms": round(res.percentile(99), 3),
                     "makespan_ms": round(res.makespan_ms, 3),
                     "gpairs_s": round(pairs / (res.makespan_ms * 1e-3) / 1e9, 3),
                     "ticks": res.ticks, "mean_batch": round(float(np.mean(res.batch_sizes)), 2),
                     "launches_per_tick": round(float(np.mean(res.launches)), 2),
                     "launches": int(np.sum(res.launches)),
                     "peak_request_bytes": res.peak_bytes, "workspace_bytes": res.fixed_bytes}
    out["batched_over_plain"] = round(out["batched"]["gpairs_s"] / out["plain"]["gpairs_s"], 3)
    torch.cuda.synchronize()
    return out


if __name__ == "__main__":
    main()
