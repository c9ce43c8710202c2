"""Host logic of the serving loop (no GPU): FIFO admission under the HBM
budget, footprint accounting and the arrival process."""
import collections

import numpy as np
import pytest

import scenes


@pytest.fixture(scope="module")
def sv():
    from paper_2506_03747_amd import serving
    return serving


def test_admission_fifo_and_budget(sv):
    adm = sv.Admission(budget_bytes=100, max_batch=3)
    sizes = [40, 30, 20, 50, 10, 200, 5]
    q = collections.deque(range(7))
    got, rej = adm.admit(q, sizes)
    assert got == [0, 1, 2] and rej == []          # batch limit
    assert adm.in_use == 90
    got, rej = adm.admit(q, sizes)
    assert got == [] and list(q) == [3, 4, 5, 6]   # head (50) does not fit: nobody overtakes it
    adm.release(40 + 30)
    got, rej = adm.admit(q, sizes)
    assert got == [3, 4, 6] and rej == [5]         # 200 > whole budget: rejected at the head
    assert not q and adm.in_use == 20 + 50 + 10 + 5
    assert adm.peak <= adm.budget
    adm.release(20 + 50 + 10 + 5)
    assert adm.in_use == 0
    with pytest.raises(RuntimeError):
        adm.release(1)


def test_admission_never_exceeds_budget_random(sv):
    rng = np.random.default_rng(3)
    sizes = rng.integers(1, 60, 500).tolist()
    adm = sv.Admission(budget_bytes=100, max_batch=8)
    q = collections.deque(range(500))
    inflight = collections.deque()
    served = []
    while q or inflight:
        got, rej = adm.admit(q, sizes)
        assert not rej
        assert adm.in_use <= 100
        if got:
            inflight.append(got)
            served.extend(got)
        if inflight and (not got or len(inflight) > 2):
            adm.release(sum(sizes[i] for i in inflight.popleft()))
    assert served == list(range(500))              # arrival order kept
    assert adm.peak <= 100 and adm.in_use == 0


def test_footprint_counts_maps_records_output(sv):
    sc = scenes.tiny(seed=3, scan=(5, 7), patches=(9, 11), n_bins=77)
    npx = 99
    b = sv.footprint_bytes(sc, with_workspace=False)
    out = 4 * 35 * 77
    assert b == 4 * npx + 4 * npx + npx + 32 * npx + 4 + out
    # the one-call workspace: 32 B of pair-loop constants per pixel, summaries, counts
    w = sv.footprint_bytes(sc) - b
    assert 32 * npx < w <= 33 * npx + 4096
    sc.mask = None
    sc.albedo = None
    assert sv.footprint_bytes(sc, with_workspace=False) == b - 5 * npx


def test_admission_pixel_cap(sv):
    adm = sv.Admission(budget_bytes=1000, max_batch=10)
    q = collections.deque(range(5))
    sizes = [1] * 5
    pixels = [40, 50, 0, 120, 30]
    got, rej = adm.admit(q, sizes, pixels=pixels, max_pixels=100)
    assert got == [0, 1, 2] and rej == [3]         # 40 + 50 + 0 <= 100; 120 alone passes the cap
    assert list(q) == [4]                          # 40 + 50 + 30 would pass it: next tick
    got, rej = adm.admit(q, sizes, pixels=pixels, max_pixels=100)
    assert got == [4] and rej == []


def test_poisson_arrivals(sv):
    a = sv.poisson_arrivals(20000, 500.0, seed=1)
    assert np.all(np.diff(a) > 0)
    assert abs(20000 / a[-1] - 500.0) < 15.0       # rate within ~4 sigma
    gaps = np.diff(a)
    assert abs(np.std(gaps) / np.mean(gaps) - 1.0) < 0.05   # exponential gaps: CV = 1
    with pytest.raises(ValueError):
        sv.poisson_arrivals(3, 0.0)


def test_server_rejects_bad_arrivals(sv):
    s = sv.Server.__new__(sv.Server)
    with pytest.raises(ValueError):
        sv.Server(mode="fast")
    s.budget, s.max_batch, s.depth, s.mode = 1 << 20, 4, 2, "batched"
    s.tick_pixels, s.fixed_bytes, s.slots, s.streams = 1 << 20, 0, [], []
    with pytest.raises(ValueError):
        sv.Server.serve(s, [scenes.tiny(seed=1)] * 2, [0.2, 0.1], staged=[None, None])


def test_admission_work_cap(sv):
    adm = sv.Admission(budget_bytes=1000, max_batch=10)
    q = collections.deque(range(5))
    sizes = [1] * 5
    work = [5.0, 3.0, 4.0, 9.0, 1.0]
    got, _ = adm.admit(q, sizes, work, max_work=8.0)
    assert got == [0, 1]                           # 5 + 3 = 8; the 4 would pass the cap
    got, _ = adm.admit(q, sizes, work, max_work=8.0)
    assert got == [2]                              # 4 + 9 > 8
    got, _ = adm.admit(q, sizes, work, max_work=8.0)
    assert got == [3]                              # first request always taken, even above the cap
    got, _ = adm.admit(q, sizes, work, max_work=8.0)
    assert got == [4]


def test_pair_count_matches_presence_rule(sv):
    sc = scenes.tiny(seed=9, scan=(3, 4), patches=(10, 12))
    sc.depth[0, 0] = np.nan
    sc.depth[1, 0] = -1.0
    sc.albedo[2, 0] = 0.0
    pres = (sc.mask != 0) & (sc.albedo > 0) & np.isfinite(sc.depth) & (sc.depth > 0)
    assert sv.pair_count(sc) == 12 * int(pres.sum())
