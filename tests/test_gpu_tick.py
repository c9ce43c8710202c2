"""Serving ticks on the GPU: a list of requests through one tick (the graph
launch, and the same operations launched eagerly) gives, for each request,
the records and count of nlos_simulate for it alone bit for bit, and its
histograms bit for bit (to 1e-6 where partial histograms meet in float
atomics); a slot's graph replayed over changing request lists, with eager
work and synchronisations between the replays, matches every time; tick
outputs match the oracle."""
import numpy as np
import pytest

import oracle
import scenes
from gpu_helpers import assert_parity, assert_parity_model, log, parity_tolerance, to_gpu

pytestmark = pytest.mark.gpu


def _req(sc):
    import paper_2506_03747_amd as nl
    depth, albedo, mask = to_gpu(sc)
    return dict(params=nl.params_of(sc), grid=sc.patch_grid, depth=depth, albedo=albedo, mask=mask)


def _empty(seed):
    sc = scenes.tiny(seed=seed, scan=(4, 4), patches=(8, 8))
    sc.mask = np.zeros_like(sc.mask)
    return sc


MIX = [
    lambda: scenes.tiny(seed=900),
    lambda: scenes.tiny(seed=901, standoff_m=0.8, n_bins=96, bin_ps=40.0),
    lambda: scenes.tiny(seed=902, cosines=False, scan=(3, 5), patches=(11, 9)),
    lambda: scenes.tiny(seed=903, fwhm_ps=0.0, scan=(9, 9), patches=(17, 17), n_bins=61),
    lambda: scenes.tiny(seed=904, scan=(2, 2), patches=(160, 160), n_bins=256, bin_ps=20.0, fwhm_ps=60.0,
                        masked=False),                                 # patches split: float atomics
    lambda: scenes.tiny(seed=905, scan=(1, 1), patches=(6, 6)),
    lambda: _empty(906),
    scenes.cfg1,
    lambda: scenes.cfg4_request(3, seed=40, max_scan=64, max_patch=65536),
    lambda: scenes.cfg4_request(7, seed=40, max_scan=64, max_patch=65536),
]


def _check_against_alone(scs, res, what):
    import torch
    import paper_2506_03747_amd as nl
    for sc, (out, rec, n) in zip(scs, res):
        prm = nl.params_of(sc)
        depth, albedo, mask = to_gpu(sc)
        out2, rec2, n2 = nl.simulate(prm, depth, sc.patch_grid, albedo, mask)
        torch.cuda.synchronize()
        k = int(n.item())
        assert k == int(n2.item()), f"{what} {sc.name}: n_active"
        assert torch.equal(rec[:k].view(torch.int32), rec2[:k].view(torch.int32)), f"{what} {sc.name}: records"
        # the tick plans its own share of the GPU, so its unit shape may
        # differ from the call alone's; the scales do not (they belong to
        # the aligned scale blocks), so the bits are the same unless either
        # plan splits the patches over workgroups (float atomics)
        # (a tick's share of the GPU is at most the call alone's, so it
        # splits only where the call alone does)
        if nl.get_plan(prm, sc.n_patch_total)["n_split"] > 1:
            e = assert_parity(out.cpu().numpy(), out2.cpu().numpy().astype(np.float64), tol=1e-6,
                              what=f"{what} {sc.name}")
            log(f"{what} {sc.name} (split): rel-L2 to the call alone {e:.2e}")
        else:
            assert torch.equal(out.view(torch.int32), out2.view(torch.int32)), f"{what} {sc.name}: histograms"


@pytest.mark.parametrize("graph", [True, False], ids=["graph", "eager"])
def test_tick_matches_simulate_alone(graph):
    import torch
    import paper_2506_03747_amd as nl
    scs = [m() for m in MIX]
    slot = nl.TickGraph(len(scs), sum(sc.n_patch_total for sc in scs), graph=graph)
    res = slot.plan([_req(sc) for sc in scs])
    slot.launch()
    torch.cuda.synchronize()
    _check_against_alone(scs, res, "graph" if graph else "eager")
    slot.close()


def test_tick_graph_replays_over_changing_lists():
    """One slot's graph, instantiated once, replayed for five different
    request lists (different counts, so different pair grids), with eager
    work on the stream and host synchronisations between the replays; every
    replay against the eager tick of the same list and the calls alone."""
    import torch
    import paper_2506_03747_amd as nl
    lists = [[0, 1, 2], [7], [3, 4, 5, 6, 8, 9], [], [9, 0, 7, 2]]
    cap_px = max(sum(MIX[i]().n_patch_total for i in ids) for ids in lists if ids)
    g = nl.TickGraph(6, cap_px, graph=True)
    e = nl.TickGraph(6, cap_px, graph=False)
    for r, ids in enumerate(lists):
        scs = [MIX[i]() for i in ids]
        log(f"replay {r}: {[sc.name for sc in scs]}")
        res_g = g.plan([_req(sc) for sc in scs])
        g.launch()
        # eager work of the program between the replays
        x = torch.randn(1 << 20, device="cuda")
        (x * 2.0).sum().item()
        res_e = e.plan([_req(sc) for sc in scs])
        e.launch()
        torch.cuda.synchronize()
        for sc, a, b in zip(scs, res_g, res_e):
            k = int(b[2].item())
            assert int(a[2].item()) == k
            assert torch.equal(a[1][:k].view(torch.int32), b[1][:k].view(torch.int32))
            if nl.get_plan(nl.params_of(sc), sc.n_patch_total)["n_split"] > 1:
                assert_parity(a[0].cpu().numpy(), b[0].cpu().numpy().astype(np.float64), tol=1e-6,
                              what=f"replay {r} {sc.name}")
            else:
                assert torch.equal(a[0].view(torch.int32), b[0].view(torch.int32)), f"replay {r} {sc.name}"
        _check_against_alone(scs, res_g, f"replay {r}")
    g.close()


def test_tick_outputs_match_oracle():
    """Every request of a tick of serving-mix requests against the oracle on
    sampled histograms, each within its own tolerance (max(1e-5, error-model
    bound))."""
    import torch
    import paper_2506_03747_amd as nl
    scs = [scenes.cfg4_request(i, seed=41, max_scan=64, max_patch=65536) for i in range(6)]
    slot = nl.TickGraph(len(scs), sum(sc.n_patch_total for sc in scs))
    res = slot.plan([_req(sc) for sc in scs])
    slot.launch()
    torch.cuda.synchronize()
    for sc, (out, _, _) in zip(scs, res):
        H = sc.n_scan
        sub = np.sort(np.random.default_rng(sc.seed).choice(H, min(H, 256), replace=False)).astype(np.int32)
        rec = oracle.patches(sc)
        ref = oracle.forward(sc, rec, subset=sub)["tau"]
        got = out.reshape(H, -1)[torch.from_numpy(sub).long().cuda()].cpu().numpy()
        tol = parity_tolerance(sc, ref, subset=sub, rec=rec)
        assert_parity_model(got, ref, tol, what=f"tick {sc.name}")
    slot.close()


def test_tick_rejects_what_it_cannot_run():
    import paper_2506_03747_amd as nl
    slot = nl.TickGraph(4, 1 << 16)
    nc = scenes.tiny(seed=910, laser=(2, 2))
    assert not nl.tick_supported(nl.params_of(nc), nc.patch_grid)
    with pytest.raises(nl.NlosError):
        slot.plan([_req(scenes.tiny(seed=911)), _req(nc)])
    win = scenes.tiny(seed=912, scan=(2, 3), patches=(24, 24), n_bins=50000, bin_ps=2.0, fwhm_ps=40.0,
                      zlo=0.5, zhi=4.0, half=2.0)
    assert not nl.tick_supported(nl.params_of(win), win.patch_grid)
    with pytest.raises(nl.NlosError):
        slot.plan([_req(win)])
    big = scenes.tiny(seed=913, scan=(2, 2), patches=(300, 300), n_bins=64)
    with pytest.raises(nl.NlosError):           # more pixels than the slot holds
        slot.plan([_req(big)])
    slot.close()
