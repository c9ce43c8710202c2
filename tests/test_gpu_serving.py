"""Serving loop on the GPU: every request gives the same result served alone
and in the mix (bit for bit, or to 1e-6 where partial histograms meet in
float atomics), every served output matches the FP64 oracle on sampled
histograms (each within its own tolerance, max(1e-5, error-model bound)),
ticks run as graph launches on overlapping streams, and the HBM budget binds
without the device memory the server allocates ever passing it."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_helpers import assert_parity, assert_parity_model, gpu_forward, log, parity_tolerance

pytestmark = pytest.mark.gpu


def _mix():
    reqs = [scenes.cfg4_request(i, seed=40, max_scan=48, max_patch=40000) for i in range(10)]
    reqs += [scenes.tiny(seed=800 + i, scan=(3 + i, 4), patches=(9 + 2 * i, 7 + i), n_bins=64 + 16 * i)
             for i in range(4)]
    # requests a tick cannot run, served through the one-call path in the mix
    reqs.append(scenes.tiny(seed=810, laser=(2, 2), standoff_m=0.5))
    reqs.append(scenes.tiny(seed=811, scan=(2, 3), patches=(24, 24), n_bins=50000, bin_ps=2.0, fwhm_ps=40.0,
                            zlo=0.5, zhi=4.0, half=2.0))
    return reqs


def _same_as_alone(r, o, what):
    import paper_2506_03747_amd as nl
    alone, _, _ = gpu_forward(r)
    if nl.get_plan(nl.params_of(r), r.n_patch_total)["n_split"] > 1:
        assert_parity(o.cpu().numpy(), alone.cpu().numpy().astype(np.float64), tol=1e-6, what=what)
    else:
        import torch
        assert torch.equal(o.view(torch.int32), alone.view(torch.int32)), what


def _oracle_sampled(r, o, what, n=64):
    H = r.n_laser * r.n_scan
    sub = np.sort(np.random.default_rng(r.seed).choice(H, min(H, n), replace=False)).astype(np.int32)
    rec = oracle.patches(r)
    ref = oracle.forward(r, rec, subset=sub)["tau"]
    got = o.cpu().numpy().reshape(H, -1)[sub]
    assert_parity_model(got, ref, parity_tolerance(r, ref, subset=sub, rec=rec), what=what)


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_same_result_alone_in_mix_and_oracle(mode):
    from paper_2506_03747_amd import serving
    reqs = _mix()
    sizes = [serving.footprint_bytes(r) for r in reqs]
    tick_px = 1 << 18
    fixed = 0 if mode == "plain" else None
    srv0 = serving.Server(budget_bytes=1 << 40, max_batch=6, depth=3, mode=mode, tick_pixels=tick_px)
    fixed = srv0.fixed_bytes
    del srv0
    budget = fixed + 3 * max(sizes)                      # admission must bind
    # the first six wait at the start (so a batched tick forms whatever the
    # GPU's speed), the rest arrive over time while ticks are in flight
    arrivals = serving.poisson_arrivals(len(reqs), 2000.0, seed=5)
    arrivals[:6] = 0.0
    log(f"serving {mode}: {len(reqs)} requests, budget {budget} B")
    srv = serving.Server(budget_bytes=budget, max_batch=6, depth=3, mode=mode, tick_pixels=tick_px)
    res = srv.serve(reqs, arrivals, keep_outputs=True)
    assert not res.rejected
    assert res.peak_bytes + res.fixed_bytes <= budget
    assert sum(res.batch_sizes) == len(reqs)
    if mode == "batched":
        assert max(res.batch_sizes) > 1 and res.ticks < len(reqs)
        assert min(res.launches) >= 1
        log(f"batched: {res.ticks} ticks, launches per tick {res.launches}")
    else:
        assert max(res.batch_sizes) == 1
    assert np.all(np.isfinite(res.latency_ms)) and np.all(res.latency_ms > 0)
    for r, o in zip(reqs, res.outputs):
        _same_as_alone(r, o, f"{mode} {r.name}")
        _oracle_sampled(r, o, f"{mode} {r.name} vs oracle")


@pytest.mark.parametrize("mode", ["batched", "plain"])
def test_device_memory_stays_within_budget(mode):
    """What the server allocates on the device while serving (maps, records,
    outputs, workspaces), measured by the allocator's peak, stays within the
    budget (its tick workspaces included)."""
    import torch
    from paper_2506_03747_amd import serving
    reqs = _mix()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    base = torch.cuda.memory_allocated()
    torch.cuda.reset_peak_memory_stats()
    sizes = [serving.footprint_bytes(r) for r in reqs]
    budget = (96 << 20) + 2 * max(sizes)
    srv = serving.Server(budget_bytes=budget, max_batch=6, depth=3, mode=mode, tick_pixels=1 << 18)
    res = srv.serve(reqs, np.zeros(len(reqs)))
    torch.cuda.synchronize()
    peak = torch.cuda.max_memory_allocated() - base
    log(f"{mode}: device peak {peak} B of budget {budget} B (requests {res.peak_bytes} B + "
        f"workspaces {res.fixed_bytes} B)")
    assert not res.rejected
    assert peak <= budget + (1 << 20)                  # the allocator rounds each block up


def test_oversized_request_rejected_others_served():
    from paper_2506_03747_amd import serving
    reqs = _mix()[:5]
    sizes = [serving.footprint_bytes(r) for r in reqs]
    big = int(np.argmax(sizes))
    srv0 = serving.Server(budget_bytes=1 << 40, max_batch=4)
    fixed = srv0.fixed_bytes
    del srv0
    budget = fixed + sorted(sizes)[-2] + 1             # everything but the largest fits
    srv = serving.Server(budget_bytes=budget, max_batch=4)
    res = srv.serve(reqs, np.zeros(len(reqs)), keep_outputs=True)
    assert res.rejected == [big]
    assert np.isnan(res.latency_ms[big]) and res.outputs[big] is None
    for i, (r, o) in enumerate(zip(reqs, res.outputs)):
        if i != big:
            _same_as_alone(r, o, r.name)
