"""Autotuner of the forward's launch plan.

For each class of problems (confocal or not, window length, number of
histograms) it forces every supported unit shape in turn through the tuning
table, times the forward operator on a seeded synthetic scene of that class
(HIP events, median of repeated launches), and keeps the fastest.  The result
is written as a JSON table that the package installs at import
(``load_tuning``); ``python -m paper_2506_03747_amd.autotune [out.json]``.

Timing only chooses among shapes the library already supports; every shape
computes the same result (the GPU tests force each one and compare them
with the oracle).
"""
from __future__ import annotations

import json
import sys

import numpy as np

from . import forward, get_plan, make_params, out_shape, patches_from_depth, reset_tuning, set_tuning

CONFOCAL_UNITS = [(1, 4, 4), (1, 4, 2), (1, 2, 2), (1, 2, 1)]
NONCONFOCAL_UNITS = [(2, 2, 2), (2, 1, 2), (1, 1, 2)]

# Classes: (confocal, t range, histogram range) and the problem each is timed
# on: window T, bin width, scan side, laser side (0: confocal).
CLASSES = []
for _t_min, _t_max, _T, _bin in [(1, 767, 512, 16.0), (768, 1535, 1024, 8.0), (1536, 4096, 2048, 4.0)]:
    for _h_min, _h_max, _ns in [(1, 2047, 32), (2048, 8191, 64), (8192, 1 << 40, 128)]:
        CLASSES.append(dict(confocal=1, t_min=_t_min, t_max=_t_max, h_min=_h_min, h_max=_h_max,
                            T=_T, bin_ps=_bin, scan=_ns, lasers=0))
    CLASSES.append(dict(confocal=0, t_min=_t_min, t_max=_t_max, h_min=1, h_max=1 << 40,
                        T=_T, bin_ps=_bin, scan=64, lasers=4))


def _scene(cls, n_patch, seed):
    """Seeded planar-ish hidden surface facing a 2 x 2 m wall, half the
    patches masked out, depths spread over the middle of the window."""
    import torch
    rng = np.random.default_rng(seed)
    reach = 299792458.0 * cls["T"] * cls["bin_ps"] * 1e-12 / 2.0      # one-way range of the window
    z = np.asarray(0.3 * reach + 0.15 * reach * rng.uniform(size=(n_patch, n_patch)), np.float32)
    mask = (rng.uniform(size=(n_patch, n_patch)) < 0.5).astype(np.uint8)
    alb = rng.uniform(0, 1, (n_patch, n_patch)).astype(np.float32)
    side = lambda n: dict(nx=n, ny=n, half_x=1.0, half_y=1.0, cx=0.0, cy=0.0)
    rec, n = patches_from_depth(torch.from_numpy(z).cuda(), side(n_patch), torch.from_numpy(alb).cuda(),
                                torch.from_numpy(mask).cuda())
    laser = side(cls["lasers"]) if cls["lasers"] else None
    prm = make_params(side(cls["scan"]), cls["T"], cls["bin_ps"], 50.0, laser=laser)
    return prm, rec, n


def _time(fn, reps=7):
    import torch
    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts))


def tune(n_patch=192, classes=CLASSES, verbose=True):
    """Time every unit per class; returns (table entries, all timings)."""
    import torch
    entries, report = [], []
    try:
        for k, cls in enumerate(classes):
            prm, rec, n = _scene(cls, n_patch, seed=1000 + k)
            out = torch.empty(out_shape(prm), dtype=torch.float32, device="cuda")
            key = {f: cls[f] for f in ("confocal", "t_min", "t_max", "h_min", "h_max")}
            best = None
            for unit in (CONFOCAL_UNITS if cls["confocal"] else NONCONFOCAL_UNITS):
                set_tuning([dict(key, tl=unit[0], tx=unit[1], ty=unit[2])])
                plan = get_plan(prm, rec.shape[0])
                if (plan["tl"], plan["tx"], plan["ty"]) != unit:
                    continue            # histograms of this unit do not fit in LDS at this window
                ms = _time(lambda: forward(prm, rec, n, out=out))
                report.append(dict(key, T=cls["T"], scan=cls["scan"], lasers=cls["lasers"], unit=list(unit),
                                   ms=ms, plan=plan))
                if verbose:
                    print(f"class {k} T={cls['T']} scan={cls['scan']}^2 lasers={cls['lasers']}^2 "
                          f"unit={unit}: {ms:.4f} ms  {plan}", flush=True)
                if best is None or ms < best[0]:
                    best = (ms, unit)
            if best:
                entries.append(dict(key, tl=best[1][0], tx=best[1][1], ty=best[1][2]))
            del out
    finally:
        reset_tuning()
    return entries, report


def main(argv=None):
    import torch
    argv = sys.argv[1:] if argv is None else argv
    out = argv[0] if argv else "tuning.json"
    entries, report = tune()
    with open(out, "w") as f:
        json.dump({"device": torch.cuda.get_device_name(0), "entries": entries, "timings": report}, f, indent=1)
    print(json.dumps(entries))


if __name__ == "__main__":
    main()
