"""HIP path against the FP64 oracle on the same seeded inputs (GPU).

Bar: bins bit-exact; every histogram within relative L2 1e-5 of the oracle
(exact zeros where the oracle's histogram is zero)."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_helpers import (assert_parity, assert_parity_model, gpu_forward, gpu_patches, guard_delta, log,
                         oracle_bins_for_records, parity_tolerance, rel_l2_rows, to_gpu)

pytestmark = pytest.mark.gpu


def _records_vs_oracle(sc):
    import torch
    patches, n_act = gpu_patches(sc)
    torch.cuda.synchronize()
    P = patches.cpu().numpy()
    n = int(n_act.item())
    rec = oracle.patches(sc)
    present = np.nonzero(rec[:, 7])[0]
    assert n == len(present)
    idx = P[:n, 7].view(np.int32)
    assert sorted(idx.tolist()) == present.tolist()       # every present pixel exactly once
    R = rec[idx]
    # canonical positions and depth: identical fp32 values
    np.testing.assert_array_equal(P[:n, 0], R[:, 0].astype(np.float32))
    np.testing.assert_array_equal(P[:n, 1], R[:, 1].astype(np.float32))
    np.testing.assert_array_equal(P[:n, 2], R[:, 2].astype(np.float32))
    np.testing.assert_allclose(P[:n, 3], R[:, 3], rtol=2e-6)
    np.testing.assert_allclose(P[:n, 4:7], R[:, 4:7], rtol=2e-6, atol=2e-7)
    return n


def _no_albedo_no_mask():
    """Maps without albedo (0.5 everywhere) and without mask: the geometry
    reads the depth map in their place and uses nothing of it."""
    import dataclasses
    sc = scenes.tiny(seed=302, patches=(40, 37), zlo=-0.1, zhi=0.6)   # some depths <= 0: absent
    return dataclasses.replace(sc, name="tiny302_plain", albedo=None, mask=None)


@pytest.mark.parametrize("make", [lambda: scenes.tiny(seed=300, patches=(13, 7)),
                                  lambda: scenes.tiny(seed=301, patches=(1, 1), masked=False),
                                  _no_albedo_no_mask,
                                  scenes.cfg1, scenes.cfg2, scenes.cfg3])
def test_records_match_oracle(make):
    sc = make()
    log(f"records {sc.name}")
    _records_vs_oracle(sc)


def _ord_images(x):
    """Order-preserving int32 images of fp32 values (negative values have
    their magnitude bits flipped), as the record summaries store them."""
    b = np.ascontiguousarray(x, np.float32).view(np.int32)
    return np.where(b >= 0, b, b ^ np.int32(0x7FFFFFFF))


@pytest.mark.parametrize("make", [lambda: scenes.tiny(seed=300, patches=(13, 7)), scenes.cfg1, scenes.cfg2])
def test_simulate_summaries_bound_their_records(make):
    """Invariant of the one-call path's record summaries (merged once per
    geometry block from wavefront reductions and one atomic per field): each
    is exactly the bounding box of its 256 consecutive records (x, y and
    depth minima and maxima, largest a, as order-preserving int32 images)
    with their count, and summaries past the last record stay empty.
    White-box: the summaries sit right after the geometry's counts in
    nlos_simulate's workspace.  The records themselves are checked against
    the oracle by test_records_match_oracle."""
    import ctypes as C
    import torch
    import paper_2506_03747_amd as nl
    from paper_2506_03747_amd._native import lib
    sc = make()
    log(f"summaries {sc.name}")
    depth, albedo, mask = to_gpu(sc)
    prm = nl.params_of(sc)
    g = nl.make_grid(sc.patch_grid)
    need, geo = C.c_size_t(0), C.c_size_t(0)
    assert lib().nlos_simulate_workspace_bytes(C.byref(prm), C.byref(g), C.byref(need)) == 0
    assert lib().nlos_patches_workspace_bytes(C.byref(g), C.byref(geo)) == 0
    ws = torch.full((need.value,), 0x5A, dtype=torch.uint8, device="cuda")   # stale bytes: every summary is rewritten
    _, rec, n = nl.simulate(prm, depth, sc.patch_grid, albedo, mask, workspace=ws)
    torch.cuda.synchronize()
    k = int(n.item())
    npx = g.nx * g.ny
    n_stats = (npx + 255) // 256
    off = (geo.value + 255) // 256 * 256
    st = ws[off:off + 32 * n_stats].cpu().numpy().view(np.int32).reshape(n_stats, 8)
    r = rec[:k].cpu().numpy()
    imax, imin = np.iinfo(np.int32).max, np.iinfo(np.int32).min
    for c in range(n_stats):
        part = r[256 * c:min(256 * (c + 1), k)]
        if len(part) == 0:
            want = [imax, imin, imax, imin, imax, imin, 0, 0]
        else:
            ox, oy, oz, oa = (_ord_images(part[:, i]) for i in range(4))
            want = [ox.min(), ox.max(), oy.min(), oy.max(), oz.min(), oa.max(), len(part), 0]
        np.testing.assert_array_equal(st[c], np.array(want, np.int32), err_msg=f"{sc.name} summary {c}")


TINY = [
    dict(seed=400),
    dict(seed=401, standoff_m=0.8),
    dict(seed=402, cosines=False),
    dict(seed=403, fwhm_ps=0.0),
    dict(seed=404, scan=(3, 5), patches=(11, 9)),
    dict(seed=405, scan=(7, 2), patches=(5, 13), standoff_m=0.4),
    dict(seed=406, scan=(9, 9), patches=(17, 17), n_bins=61),            # T not a multiple of 4
    dict(seed=407, scan=(1, 1), patches=(6, 6)),
    dict(seed=408, laser=(2, 2), standoff_m=0.6),
    dict(seed=409, laser=(3, 1), scan=(3, 4), standoff_m=0.0, cosines=False),
    dict(seed=410, laser=(1, 1), scan=(5, 3), fwhm_ps=0.0),
    dict(seed=411, laser=(5, 3), scan=(3, 3), patches=(9, 10), standoff_m=1.1),
]


@pytest.mark.parametrize("kw", TINY, ids=[str(k["seed"]) for k in TINY])
def test_tiny_parity(kw):
    sc = scenes.tiny(**kw)
    log(f"tiny {kw}")
    tau, _, _ = gpu_forward(sc)
    ref = oracle.forward(sc)["tau"]
    assert_parity(tau.cpu().numpy(), ref, what=sc.name)


@pytest.mark.parametrize("kw", TINY[:6] + TINY[8:], ids=[str(k["seed"]) for k in TINY[:6] + TINY[8:]])
def test_tiny_bins_exact(kw):
    import torch
    import paper_2506_03747_amd as nl
    sc = scenes.tiny(**kw)
    log(f"bins {kw}")
    patches, n_act = gpu_patches(sc)
    bins = nl.debug_bins(nl.params_of(sc), patches, n_act)
    torch.cuda.synchronize()
    n = int(n_act.item())
    P = patches.cpu().numpy()
    ref = oracle_bins_for_records(sc, P, n)
    got = bins.cpu().numpy()
    np.testing.assert_array_equal(got[:, :n], ref)
    assert np.all(got[:, n:] == np.iinfo(np.int32).min)


def test_cfg1_full():
    sc = scenes.cfg1()
    log("cfg1")
    tau, _, _ = gpu_forward(sc)
    ref = oracle.forward(sc)["tau"]
    e = assert_parity(tau.cpu().numpy(), ref, what="cfg1")
    log(f"cfg1 worst rel-L2 {e:.3e}")


def test_cfg2_full():
    sc = scenes.cfg2()
    log("cfg2")
    tau, _, _ = gpu_forward(sc)
    ref = oracle.forward(sc)["tau"]
    e = assert_parity(tau.cpu().numpy(), ref, what="cfg2")
    log(f"cfg2 worst rel-L2 {e:.3e}")


def test_cfg5_full():
    sc = scenes.cfg5()
    log("cfg5")
    tau, _, _ = gpu_forward(sc)
    ref = oracle.forward(sc)["tau"]
    e = assert_parity(tau.cpu().numpy(), ref, what="cfg5")
    log(f"cfg5 worst rel-L2 {e:.3e}")


def _cfg3_subset(tau, H, n_rand=4096, n_weak=64):
    """4096 seeded histograms and the 64 weakest non-empty ones (weakest by
    the GPU's output: the choice of cases only, every value is checked
    against the oracle)."""
    import torch
    rng = np.random.default_rng(33)
    rand = rng.choice(H, n_rand, replace=False)
    norms = tau.reshape(H, -1).double().norm(dim=1)
    norms[norms == 0] = float("inf")
    weakest = torch.topk(norms, n_weak, largest=False).indices.cpu().numpy()
    return np.unique(np.concatenate([rand, weakest])).astype(np.int32), weakest


def _check_cfg3(tau, sc, what):
    """cfg3 (64 lasers x 128^2 detectors x T = 2048, 8.6 GB): sampled
    histograms against the oracle, each within its own tolerance
    max(1e-5, error-model bound): the bound exceeds 1e-5 only where a
    histogram is made of a few pairs seen nearly edge-on, whose fp32 cosines
    are ill-conditioned (or far weaker than their unit's fixed-point bound)."""
    import torch
    H = sc.n_laser * sc.n_scan
    sub, weakest = _cfg3_subset(tau, H)
    got = tau.reshape(H, -1)[torch.from_numpy(sub).long().cuda()].cpu().numpy()
    rec = oracle.patches(sc)
    ref = oracle.forward(sc, rec, subset=sub)["tau"]
    tol = parity_tolerance(sc, ref, subset=sub, rec=rec)
    e, ratio, loose = assert_parity_model(got, ref, tol, what=what)
    in_w = np.isin(sub, weakest)
    log(f"{what}: the 64 weakest: worst rel-L2 {rel_l2_rows(got[in_w], ref[in_w]).max():.3e}")
    return e


def test_cfg3_sampled():
    import torch
    sc = scenes.cfg3()
    log("cfg3")
    tau, _, _ = gpu_forward(sc)
    _check_cfg3(tau, sc, "cfg3 forward")
    del tau
    torch.cuda.empty_cache()


@pytest.mark.parametrize("name,n_hist", [("cfg1", None), ("cfg2", 256), ("cfg3", 128)])
def test_bins_exact_configs(name, n_hist):
    import torch
    import paper_2506_03747_amd as nl
    sc = scenes.by_name(name)
    log(f"bins {name}")
    patches, n_act = gpu_patches(sc)
    prm = nl.params_of(sc)
    H = nl.n_histograms(prm)
    if n_hist is None:
        sub = np.arange(H, dtype=np.int32)
    else:
        sub = np.sort(np.random.default_rng(7).choice(H, n_hist, replace=False)).astype(np.int32)
    n = int(n_act.item())
    # the GPU export covers every histogram; keep memory modest on the big ones
    rows = []
    Pn = patches.cpu().numpy()
    if H * patches.shape[0] <= (1 << 28):
        bins = nl.debug_bins(prm, patches, n_act)
        torch.cuda.synchronize()
        got = bins[torch.from_numpy(sub).long().cuda()].cpu().numpy()
        del bins
    else:
        # cfg3: pass a record subset of the same patches through fewer histograms is not
        # possible (H is fixed), so split the records instead
        step = max(1, (1 << 28) // H)
        for s0 in range(0, n, step):
            part = patches[s0:min(n, s0 + step)].contiguous()
            b = nl.debug_bins(prm, part, None)
            torch.cuda.synchronize()
            rows.append(b[torch.from_numpy(sub).long().cuda()].cpu().numpy())
            del b
        got = np.concatenate(rows, axis=1)
    ref = oracle_bins_for_records(sc, Pn, n, subset=sub)
    np.testing.assert_array_equal(got[:, :n], ref)


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3"])
def test_guard_band_holds(name):
    """The fp32 arrival stays within half the guard width of the fp64 one for
    every pair at or before the window end: the fast path's bins are safe."""
    import torch
    import paper_2506_03747_amd as nl
    sc = scenes.by_name(name)
    log(f"guard {name}")
    patches, n_act = gpu_patches(sc)
    n = int(n_act.item())
    prm = nl.params_of(sc)
    H = nl.n_histograms(prm)
    cap = max(1, (1 << 26) // H)
    part = patches[: min(n, cap)].contiguous()
    _, uf, ue = nl.debug_bins(prm, part, None, want_u=True)
    torch.cuda.synchronize()
    near = ue <= sc.n_bins + 1
    err = (uf - ue).abs()[near].max().item()
    d = guard_delta(sc.n_bins)
    log(f"{name}: max |u32 - u64| = {err:.3e} bins, guard {d:.3e}")
    assert err <= 0.5 * d


def test_empty_scene():
    sc = scenes.tiny(seed=500, scan=(4, 4), patches=(8, 8))
    sc.mask = np.zeros_like(sc.mask)
    tau, _, n_act = gpu_forward(sc)
    assert int(n_act.item()) == 0
    assert not tau.cpu().numpy().any()


@pytest.mark.parametrize("n", [1, 63, 64, 65, 127, 129, 1023, 1025])
def test_record_counts_around_chunks(n):
    """Record counts on both sides of the pair loop's 64-record chunks (a
    wavefront holds two, the next one's records loaded ahead): a mask with
    exactly n present pixels."""
    sc = scenes.tiny(seed=520 + n, scan=(5, 4), patches=(40, 40), n_bins=128)
    rng = np.random.default_rng(n)
    m = np.zeros(40 * 40, np.uint8)
    m[rng.choice(40 * 40, n, replace=False)] = 1
    sc.mask = m.reshape(40, 40)
    log(f"records {n}")
    tau, _, n_act = gpu_forward(sc)
    assert int(n_act.item()) == n
    ref = oracle.forward(sc)["tau"]
    assert ref.any()
    assert_parity(tau.cpu().numpy(), ref, what=f"n={n}")


def test_without_n_active_pointer():
    sc = scenes.tiny(seed=501, scan=(5, 5), patches=(12, 12), standoff_m=0.3)
    tau, _, _ = gpu_forward(sc, use_n_active=False)
    assert_parity(tau.cpu().numpy(), oracle.forward(sc)["tau"], what="no n_active")


def test_single_bin_window():
    sc = scenes.tiny(seed=502, scan=(3, 3), patches=(10, 10), n_bins=1, bin_ps=5000.0, fwhm_ps=0.0)
    tau, _, _ = gpu_forward(sc)
    ref = oracle.forward(sc)["tau"]
    assert ref.any()
    assert_parity(tau.cpu().numpy(), ref, what="T=1")


@pytest.mark.parametrize("fwhm_ps", [40.0, 20.0], ids=["radius17", "radius9"])
def test_time_windows(fwhm_ps):
    """A histogram longer than LDS: the time axis is split over workgroups,
    one row each.  Radius 17 takes the flush's generic tap loop; radius 9
    (taps padded to 12) deals the row's jitter segments to all 16
    wavefronts of the workgroup."""
    sc = scenes.tiny(seed=503, scan=(2, 3), patches=(24, 24), n_bins=50000, bin_ps=2.0,
                     fwhm_ps=fwhm_ps, zlo=0.5, zhi=4.0, half=2.0)
    tau, _, _ = gpu_forward(sc)
    ref = oracle.forward(sc)["tau"]
    assert_parity(tau.cpu().numpy(), ref, what="time windows")


def _sphere_cap_scene():
    """16 x 16 confocal scan points; a 128 x 128 depth map on the sphere of
    radius R around scan point (8, 8), R chosen so that every pair of that
    scan point arrives 3e-4 bins below bin 500 (fp32 coordinates move it by
    about 4e-5 bins)."""
    c = 299792458.0
    bin_ps, T, half_w, half_p, n_p = 8.0, 1024, 0.5, 0.3, 128
    canon = lambda half, n: (-half + (np.arange(n) + 0.5) * (2.0 * half / n)).astype(np.float32).astype(np.float64)
    x0 = canon(half_w, 16)[8]
    xs = canon(half_p, n_p)
    R = (500.0 - 3e-4) * c * bin_ps * 1e-12 / 2.0
    dx2 = (xs[:, None] - x0) ** 2 + (xs[None, :] - x0) ** 2
    z = np.sqrt(R * R - dx2).astype(np.float32)
    rng = np.random.default_rng(512)
    albedo = rng.uniform(0.5, 1.0, (n_p, n_p)).astype(np.float32)
    return scenes.Scene("sphere_cap", scenes.grid(16, 16, half_w), None, scenes.grid(n_p, n_p, half_p), z, albedo,
                        None, standoff_m=0.0, bin_ps=bin_ps, n_bins=T, fwhm_ps=40.0, seed=512)


def test_guard_queue_overflow_moves_pairs():
    """Every pair of one scan point lies within the guard band just above a
    bin edge in fp32 and one bin lower in fp64: each is queued and moved, and
    with 4096 such pairs per workgroup against 16 wavefronts x 128 queue
    entries, the queues overflow, so the in-place correction runs too.  Checked against
    the oracle through the two-call path (raw records) and the one-call path
    (re-binning from the pair-loop constants)."""
    import torch
    import paper_2506_03747_amd as nl
    sc = _sphere_cap_scene()
    rec = oracle.patches(sc)
    ref = oracle.forward(sc, rec)["tau"]
    bins = oracle.forward(sc, rec, subset=np.array([8 * 16 + 8]), want_tau=False, want_bins=True)["bins"][0]
    assert np.all(bins == 499), "every pair of the centre scan point is in bin 499 in fp64"
    assert 500.0 - 3e-4 + guard_delta(sc.n_bins) < 500.0 + 2 * guard_delta(sc.n_bins)
    tol = parity_tolerance(sc, ref, rec=rec)
    # a workgroup's share of the records exceeds its 16 x 128 queue entries
    plan = nl.get_plan(nl.params_of(sc), sc.n_patch_total)
    assert sc.n_patch_total / plan["n_split"] > 16 * 128, plan
    two, _, _ = gpu_forward(sc)
    depth, albedo, mask = to_gpu(sc)
    one, _, _ = nl.simulate(nl.params_of(sc), depth, sc.patch_grid, albedo, mask)
    torch.cuda.synchronize()
    for what, tau in (("two-call", two), ("one-call", one)):
        got = tau.cpu().numpy().reshape(-1, sc.n_bins)
        assert_parity_model(got, ref, tol, what=f"sphere cap {what}")
        # (the jitter is symmetric: the centre histogram peaks at its pairs' bin)
        assert int(np.argmax(got[8 * 16 + 8])) == 499, f"{what}: the centre histogram's pairs left bin 499"


def test_patch_split_many_patches_few_scan_points():
    """Few histograms, many patches: patches are split over workgroups and
    the partial histograms combined with float atomics."""
    sc = scenes.tiny(seed=504, scan=(2, 2), patches=(160, 160), n_bins=256, bin_ps=20.0,
                     fwhm_ps=60.0, masked=False)
    tau, _, _ = gpu_forward(sc)
    assert_parity(tau.cpu().numpy(), oracle.forward(sc)["tau"], what="split")


def test_side_stream():
    import torch
    sc = scenes.tiny(seed=505, scan=(6, 6), patches=(20, 20), standoff_m=0.5)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        tau, _, _ = gpu_forward(sc, stream=s)
    s.synchronize()
    assert_parity(tau.cpu().numpy(), oracle.forward(sc)["tau"], what="side stream")


def near_edge_depths(n, half, bin_ps, seed):
    """Depth map whose fp64 arrivals (scan point at the origin) lie within a
    few 1e-5 bins of a bin edge: for each pixel solve for the depth of an
    exact integer arrival, then take the closest of the nearby fp32 values."""
    rng = np.random.default_rng(seed)
    inv = 1.0 / (299792458.0 * (bin_ps * 1e-12))
    xs = (-half + (np.arange(n) + 0.5) * (2 * half / n)).astype(np.float32).astype(np.float64)
    depth = np.zeros((n, n), np.float32)
    for i in range(n):
        for j in range(n):
            lat2 = xs[i] ** 2 + xs[j] ** 2
            k = int(rng.integers(int(2 * inv * np.sqrt(lat2 + 0.3 ** 2)) + 1, int(2 * inv * 0.95)))
            z = np.sqrt((k / (2 * inv)) ** 2 - lat2)
            best, bd = None, 1.0
            for t in range(-16, 17):
                zc = np.float32(z * (1 + t * 2.0 ** -24))
                r = np.sqrt((xs[i] * xs[i] + xs[j] * xs[j]) + float(zc) * float(zc))
                u = (r + r) * inv
                d = abs(u - round(u))
                if d < bd:
                    best, bd = zc, d
            depth[i, j] = best
    return depth


def test_near_edge_arrivals():
    """Every pair's fp64 arrival lies within ~1e-4 bins of a bin edge: all of
    them go through the guard band and the fp64 re-binning."""
    import torch
    import paper_2506_03747_amd as nl
    n = 32
    sc = scenes.tiny(seed=506, scan=(1, 1), patches=(n, n), n_bins=1024, bin_ps=10.0, half=0.5,
                     masked=False, fwhm_ps=50.0)
    sc.depth = near_edge_depths(n, 0.5, 10.0, 506)
    sc.relay = scenes.grid(1, 1, 0.5)
    patches, n_act = gpu_patches(sc)
    bins, uf, ue = nl.debug_bins(nl.params_of(sc), patches, n_act, want_u=True)
    torch.cuda.synchronize()
    k = int(n_act.item())
    u = ue.cpu().numpy()[:, :k]
    assert np.abs(u - np.round(u)).max() < 1e-4
    ref = oracle_bins_for_records(sc, patches.cpu().numpy(), k)
    np.testing.assert_array_equal(bins.cpu().numpy()[:, :k], ref)
    tau, _, _ = gpu_forward(sc)
    assert_parity(tau.cpu().numpy(), oracle.forward(sc)["tau"], what="near edge")


def test_repeatable_within_tolerance():
    sc = scenes.cfg1()
    a, _, _ = gpu_forward(sc)
    b, _, _ = gpu_forward(sc)
    assert_parity(a.cpu().numpy(), b.cpu().numpy().astype(np.float64), tol=1e-6, what="repeat")


@pytest.mark.parametrize("make", [scenes.cfg1, scenes.cfg2, scenes.cfg3,
                                  lambda: scenes.tiny(seed=510, scan=(2, 2), patches=(160, 160), n_bins=256,
                                                      bin_ps=20.0, fwhm_ps=60.0, masked=False),
                                  lambda: scenes.tiny(seed=511, scan=(2, 3), patches=(24, 24), n_bins=50000,
                                                      bin_ps=2.0, fwhm_ps=40.0, zlo=0.5, zhi=4.0, half=2.0)],
                         ids=["cfg1", "cfg2", "cfg3", "split", "windows"])
def test_simulate_equals_two_calls(make):
    """One call (geometry merging the record summaries + forward) gives the
    records and count of the two calls bit for bit, and -- the summaries
    covering the same 256-record blocks, so the fixed-point scales are the
    same -- the same histograms bit for bit.  Where patches are split over
    workgroups the partial histograms meet in float atomics of no fixed
    order: there the two agree to 1e-6."""
    import torch
    import paper_2506_03747_amd as nl
    sc = make()
    log(f"simulate {sc.name}")
    depth, albedo, mask = to_gpu(sc)
    prm = nl.params_of(sc)
    out, rec, n = nl.simulate(prm, depth, sc.patch_grid, albedo, mask)
    rec2, n2 = nl.patches_from_depth(depth, sc.patch_grid, albedo, mask, cosines=sc.cosines)
    out2 = nl.forward(prm, rec2, n2)
    torch.cuda.synchronize()
    k = int(n.item())
    assert k == int(n2.item())
    np.testing.assert_array_equal(rec[:k].cpu().numpy().view(np.uint32), rec2[:k].cpu().numpy().view(np.uint32))
    del rec, rec2
    split = nl.get_plan(prm, sc.n_patch_total)["n_split"] > 1
    if not split:
        same = bool(torch.equal(out.view(torch.int32), out2.view(torch.int32)))
        log(f"simulate {sc.name}: bitwise equal {same}")
        assert same, "one call and two calls differ"
    else:
        got = out.cpu().numpy()
        ref = out2.cpu().numpy().astype(np.float64)
        e = assert_parity(got, ref, tol=1e-6, what=f"simulate {sc.name} (split)")
        log(f"simulate {sc.name} (split): worst rel-L2 {e:.3e}")


@pytest.mark.parametrize("name", ["cfg1", "cfg2", "cfg3"])
def test_simulate_matches_oracle(name):
    """The benchmarked one-call path against the oracle: cfg1 and cfg2 in
    full at 1e-5 per histogram, cfg3 on 4096 seeded histograms plus its 64
    weakest, each within its own tolerance."""
    import torch
    import paper_2506_03747_amd as nl
    sc = scenes.by_name(name)
    log(f"simulate vs oracle {name}")
    depth, albedo, mask = to_gpu(sc)
    prm = nl.params_of(sc)
    out, rec, n = nl.simulate(prm, depth, sc.patch_grid, albedo, mask)
    torch.cuda.synchronize()
    if name == "cfg3":
        _check_cfg3(out, sc, "cfg3 simulate")
        del out
        torch.cuda.empty_cache()
    else:
        ref = oracle.forward(sc)["tau"]
        e = assert_parity(out.cpu().numpy(), ref, what=f"{name} simulate")
        log(f"{name} simulate: worst rel-L2 {e:.3e}")


def test_evaluated_pairs_cover_the_window():
    """The evaluated-pair count of the one-call path: every pair that lands
    in the window is evaluated (the cull is safe), and no more pairs than
    (histograms x records) are."""
    import torch
    import paper_2506_03747_amd as nl
    sc = scenes.cfg2()
    depth, albedo, mask = to_gpu(sc)
    prm = nl.params_of(sc)
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    out, rec, n = nl.simulate(prm, depth, sc.patch_grid, albedo, mask, evaluated_pairs=cnt)
    torch.cuda.synchronize()
    ev = int(cnt.item())
    in_window = int(oracle.error_model(sc)["count"].sum())
    total = sc.n_scan * int(n.item())
    log(f"evaluated {ev} of {total} pairs ({ev / total:.3f}); in the window {in_window}")
    assert in_window <= ev <= total


def test_simulate_empty_scene():
    import torch
    import paper_2506_03747_amd as nl
    sc = scenes.tiny(seed=512, scan=(4, 4), patches=(8, 8))
    sc.mask = np.zeros_like(sc.mask)
    depth, albedo, mask = to_gpu(sc)
    out, _, n = nl.simulate(nl.params_of(sc), depth, sc.patch_grid, albedo, mask)
    torch.cuda.synchronize()
    assert int(n.item()) == 0 and not out.cpu().numpy().any()


def test_large_map_uses_scan_path():
    """A depth map of more than 4096 enumeration blocks of 256 pixels (1056 x
    1024 pixels): block offsets come from the scan kernel; every present pixel
    appears exactly once and the one-call path agrees with the two calls."""
    import torch
    import paper_2506_03747_amd as nl
    rng = np.random.default_rng(77)
    nx, ny = 1056, 1024
    depth = rng.uniform(0.3, 0.6, (nx, ny)).astype(np.float32)
    mask = (rng.uniform(size=(nx, ny)) < 0.3).astype(np.uint8)
    grid = scenes.grid(nx, ny, 0.5)
    d, m = torch.from_numpy(depth).cuda(), torch.from_numpy(mask).cuda()
    rec, n = nl.patches_from_depth(d, grid, None, m)
    torch.cuda.synchronize()
    k = int(n.item())
    assert k == int(mask.sum())
    idx = np.sort(rec[:k].cpu().numpy()[:, 7].view(np.int32))
    np.testing.assert_array_equal(idx, np.nonzero(mask.ravel())[0])
    prm = nl.make_params(scenes.grid(2, 2, 0.5), 64, 50.0, 120.0)
    out, rec1, n1 = nl.simulate(prm, d, grid, None, m)
    out2 = nl.forward(prm, rec, n)
    torch.cuda.synchronize()
    assert int(n1.item()) == k
    assert_parity(out.cpu().numpy(), out2.cpu().numpy().astype(np.float64), tol=1e-6, what="large map")
