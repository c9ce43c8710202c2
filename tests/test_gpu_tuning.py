"""Every unit shape the autotuner may choose, forced through the tuning table,
against the FP64 oracle (GPU): the table changes speed, never the result."""
import pytest

import oracle
import scenes
from gpu_helpers import assert_parity, gpu_forward, log

pytestmark = pytest.mark.gpu

CONF_UNITS = [(1, 4, 4), (1, 4, 2), (1, 2, 2), (1, 2, 1), (1, 1, 1)]
NC_UNITS = [(2, 2, 2), (2, 1, 2), (1, 1, 2), (1, 1, 1)]

CASES = [
    ("cfg1", scenes.cfg1, CONF_UNITS),
    ("ragged", lambda: scenes.tiny(seed=404, scan=(3, 5), patches=(11, 9)), CONF_UNITS),
    ("laser", lambda: scenes.tiny(seed=408, laser=(2, 2), standoff_m=0.6), NC_UNITS),
    ("laser_ragged", lambda: scenes.tiny(seed=411, laser=(5, 3), scan=(3, 3), patches=(9, 10), standoff_m=1.1),
     NC_UNITS),
]


@pytest.mark.parametrize("name,make,units", CASES, ids=[c[0] for c in CASES])
def test_forced_units_match_oracle(name, make, units):
    import torch
    import paper_2506_03747_amd as nl
    sc = make()
    prm = nl.params_of(sc)
    ref = oracle.forward(sc)["tau"]
    conf = 0 if sc.laser is not None else 1
    seen = set()
    try:
        for unit in units:
            nl.set_tuning([dict(confocal=conf, t_min=1, t_max=1 << 20, h_min=1, h_max=1 << 40,
                                tl=unit[0], tx=unit[1], ty=unit[2])])
            n_rec = int(sc.patch_grid["nx"]) * int(sc.patch_grid["ny"])
            plan = nl.get_plan(prm, n_rec)
            got_unit = (plan["tl"], plan["tx"], plan["ty"])
            log(f"tuning {name} forced {unit} -> {plan}")
            if got_unit != unit:
                continue                       # does not fit in LDS at this window
            seen.add(unit)
            tau, _, _ = gpu_forward(sc)
            torch.cuda.synchronize()
            assert_parity(tau.cpu().numpy(), ref, what=f"{name} unit {unit}")
    finally:
        nl.reset_tuning()
    assert len(seen) >= 2, seen
