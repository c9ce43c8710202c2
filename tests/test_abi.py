"""The C-ABI library without a GPU: it loads, exports every entry point the
header declares, its structs have the header's layout, and host-side argument
checks give the documented codes before anything touches a device."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nlos.h")


@pytest.fixture(scope="module")
def nat():
    from paper_2506_03747_amd import _native
    _native.lib()
    return _native


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(nlos_\w+)\s*\(", src, re.M)))


def test_exports_every_declared_symbol(nat):
    names = declared_functions()
    assert len(names) == 34, names
    for n in names:
        assert hasattr(nat.lib(), n), n
    bound = {s[0] for s in nat.SIGNATURES}
    assert bound == set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", nat.LIB_PATH], capture_output=True, text=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, re.M), n


def test_version_and_strerror(nat):
    L = nat.lib()
    assert L.nlos_abi_version() == 2
    for code, text in ((0, "ok"), (-1, "invalid argument"), (-2, "workspace too small"),
                       (-3, "HIP runtime error"), (-4, "no usable GPU"), (7, "unknown error")):
        assert nat.strerror(code) == text


def test_struct_layout_matches_header(nat, tmp_path):
    """sizeof / offsetof from a C compiler reading the header itself."""
    prog = tmp_path / "lay.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "nlos.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                    'sizeof(nlos_grid), offsetof(nlos_grid, half_x), offsetof(nlos_grid, cy),'
                    'sizeof(nlos_params), offsetof(nlos_params, laser), offsetof(nlos_params, standoff_m),'
                    'offsetof(nlos_params, n_bins), offsetof(nlos_params, flags), offsetof(nlos_params, fwhm_ps));'
                    'return 0;}\n')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    G, P = nat.Grid, nat.Params
    want = [C.sizeof(G), G.half_x.offset, G.cy.offset, C.sizeof(P), P.laser.offset, P.standoff_m.offset,
            P.n_bins.offset, P.flags.offset, P.fwhm_ps.offset]
    assert got == want


def test_request_struct_layout_matches_header(nat, tmp_path):
    prog = tmp_path / "req.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "nlos.h"\n'
                    'int main(void){printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\\n",'
                    'sizeof(nlos_depth_request), offsetof(nlos_depth_request, depth),'
                    'offsetof(nlos_depth_request, albedo), offsetof(nlos_depth_request, mask),'
                    'offsetof(nlos_depth_request, flags), offsetof(nlos_depth_request, patches),'
                    'offsetof(nlos_depth_request, n_active),'
                    'sizeof(nlos_request), offsetof(nlos_request, patches), offsetof(nlos_request, n_patches),'
                    'offsetof(nlos_request, n_active), offsetof(nlos_request, out), offsetof(nlos_request, params));'
                    'return 0;}\n')
    exe = tmp_path / "req"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    D, R = nat.DepthRequest, nat.Request
    want = [C.sizeof(D), D.depth.offset, D.albedo.offset, D.mask.offset, D.flags.offset, D.patches.offset,
            D.n_active.offset, C.sizeof(R), R.patches.offset, R.n_patches.offset, R.n_active.offset,
            R.out.offset, R.params.offset]
    assert got == want


def test_probe_struct_layout_matches_header(nat, tmp_path):
    prog = tmp_path / "probe.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "nlos.h"\n'
                    'int main(void){printf("%zu %zu %zu\\n", sizeof(nlos_probe), offsetof(nlos_probe, forward_mark),'
                    'offsetof(nlos_probe, evaluated_pairs)); return 0;}\n')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True).stdout.split()]
    Pr = nat.Probe
    assert got == [C.sizeof(Pr), Pr.forward_mark.offset, Pr.evaluated_pairs.offset]


def test_batched_checks(nat):
    """Host-side checks of the batched calls: sizes, a bad request rejects the
    whole call, a short workspace or table gives NLOS_ENOSPC, n = 0 is a no-op."""
    L = nat.lib()
    reqs = (nat.Request * 3)()
    for i in range(3):
        reqs[i] = nat.Request(_params(nat, n_bins=64 * (i + 1)), 0x10000, 1000 * (i + 1), None, 0x20000)
    tb, wb = C.c_size_t(0), C.c_size_t(0)
    assert L.nlos_forward_batched_sizes(reqs, 3, C.byref(tb), C.byref(wb)) == 0
    assert tb.value >= 3 * 1024 and wb.value > tb.value   # argument table, then record summaries
    assert tb.value % 256 == 0
    assert L.nlos_forward_batched(reqs, 3, None, 0, FAKE, wb.value - 1, None) == nat.NLOS_ENOSPC
    table = (C.c_ubyte * tb.value)()
    assert L.nlos_forward_batched(reqs, 3, table, tb.value - 1, FAKE, wb.value, None) == nat.NLOS_ENOSPC
    assert L.nlos_forward_batched(reqs, 3, table, tb.value, None, wb.value, None) == nat.NLOS_EINVAL
    assert L.nlos_forward_batched(reqs, 0, None, 0, None, 0, None) == 0
    assert L.nlos_forward_batched(None, 2, None, 0, FAKE, 1 << 30, None) == nat.NLOS_EINVAL
    reqs[1].params.bin_ps = 0.0
    assert L.nlos_forward_batched_sizes(reqs, 3, C.byref(tb), C.byref(wb)) == nat.NLOS_EINVAL
    assert L.nlos_forward_batched(reqs, 3, None, 0, FAKE, 1 << 30, None) == nat.NLOS_EINVAL
    reqs[1].params.bin_ps = 16.0
    reqs[2].out = None
    assert L.nlos_forward_batched(reqs, 3, None, 0, FAKE, 1 << 30, None) == nat.NLOS_EINVAL

    g = nat.Grid(64, 64, 0.5, 0.5, 0.0, 0.0)
    maps = (nat.DepthRequest * 2)()
    maps[0] = nat.DepthRequest(g, 0x10000, None, None, 1, 0x20000, 0x30000)
    maps[1] = nat.DepthRequest(nat.Grid(300, 17, 0.5, 0.5, 0.0, 0.0), 0x10000, None, None, 1, 0x20000, 0x30000)
    assert L.nlos_patches_batched_sizes(maps, 2, C.byref(tb), C.byref(wb)) == 0
    assert wb.value > tb.value
    assert L.nlos_patches_batched(maps, 2, None, 0, FAKE, wb.value - 1, None) == nat.NLOS_ENOSPC
    assert L.nlos_patches_batched(maps, 0, None, 0, None, 0, None) == 0
    maps[1].flags = 4
    assert L.nlos_patches_batched(maps, 2, None, 0, FAKE, 1 << 30, None) == nat.NLOS_EINVAL


def _params(nat, **kw):
    g = nat.Grid(4, 4, 0.5, 0.5, 0.0, 0.0)
    p = nat.Params(g, nat.Grid(0, 0, 0, 0, 0, 0), 0.0, 16.0, 64, nat.NLOS_F_COSINES, 70.0)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


FAKE = C.c_void_p(0x10000)   # aligned, never dereferenced: checks fail first


@pytest.mark.parametrize("field,value", [
    ("bin_ps", 0.0), ("bin_ps", -1.0), ("bin_ps", float("nan")), ("n_bins", 0), ("n_bins", (1 << 22) + 1),
    ("standoff_m", -0.1), ("fwhm_ps", -1.0), ("flags", 2), ("fwhm_ps", 1e9)])
def test_forward_rejects_bad_params(nat, field, value):
    p = _params(nat, **{field: value})
    rc = nat.lib().nlos_forward(C.byref(p), FAKE, 16, None, FAKE, FAKE, 1 << 20, None)
    assert rc == nat.NLOS_EINVAL


def test_forward_rejects_bad_buffers(nat):
    L = nat.lib()
    p = _params(nat)
    assert L.nlos_forward(None, FAKE, 16, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_EINVAL
    assert L.nlos_forward(C.byref(p), None, 16, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_EINVAL
    assert L.nlos_forward(C.byref(p), FAKE, 16, None, None, FAKE, 1 << 20, None) == nat.NLOS_EINVAL
    assert L.nlos_forward(C.byref(p), C.c_void_p(0x10004), 16, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_EINVAL
    assert L.nlos_forward(C.byref(p), FAKE, -1, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_EINVAL
    assert L.nlos_forward(C.byref(p), FAKE, (1 << 24) + 1, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_EINVAL
    bad_grid = _params(nat)
    bad_grid.relay.nx = 0
    assert L.nlos_forward(C.byref(bad_grid), FAKE, 16, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_EINVAL
    half_laser = _params(nat)
    half_laser.laser.nx = 2   # ny = 0: neither confocal nor a valid laser grid
    assert L.nlos_forward(C.byref(half_laser), FAKE, 16, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_EINVAL


def test_forward_workspace(nat):
    L = nat.lib()
    p = _params(nat)
    need = C.c_size_t(0)
    assert L.nlos_forward_workspace_bytes(C.byref(p), 5000, C.byref(need)) == 0
    assert need.value >= 20 * 32         # one 32-byte summary per 256 records (+ planned pairs)
    assert L.nlos_forward(C.byref(p), FAKE, 5000, None, FAKE, FAKE, need.value - 1, None) == nat.NLOS_ENOSPC
    assert L.nlos_forward(C.byref(p), FAKE, 5000, None, FAKE, None, need.value, None) == nat.NLOS_EINVAL
    assert L.nlos_forward(C.byref(p), FAKE, 5000, None, FAKE, C.c_void_p(0x10008), need.value,
                          None) == nat.NLOS_EINVAL   # misaligned workspace


def test_patches_checks(nat):
    L = nat.lib()
    g = nat.Grid(64, 64, 0.5, 0.5, 0.0, 0.0)
    need = C.c_size_t(0)
    assert L.nlos_patches_workspace_bytes(C.byref(g), C.byref(need)) == 0
    assert need.value >= 8
    assert L.nlos_patches_from_depth(C.byref(g), FAKE, None, None, 1, FAKE, FAKE, FAKE, need.value - 1,
                                     None) == nat.NLOS_ENOSPC
    assert L.nlos_patches_from_depth(C.byref(g), None, None, None, 1, FAKE, FAKE, FAKE, need.value,
                                     None) == nat.NLOS_EINVAL
    assert L.nlos_patches_from_depth(C.byref(g), FAKE, None, None, 4, FAKE, FAKE, FAKE, need.value,
                                     None) == nat.NLOS_EINVAL
    big = nat.Grid(8192, 4096, 0.5, 0.5, 0.0, 0.0)   # 2^25 pixels > limit
    assert L.nlos_patches_from_depth(C.byref(big), FAKE, None, None, 1, FAKE, FAKE, FAKE, 1 << 30,
                                     None) == nat.NLOS_EINVAL


def test_debug_bins_limit(nat):
    p = _params(nat)
    p.relay.nx = p.relay.ny = 4096
    rc = nat.lib().nlos_debug_bins(C.byref(p), FAKE, 1 << 20, None, FAKE, None, None, None)
    assert rc == nat.NLOS_EINVAL


def _gpu_present():
    try:
        import torch
        return torch.cuda.device_count() > 0
    except Exception:   # noqa: BLE001
        return False


@pytest.mark.skipif(_gpu_present(), reason="checks the no-device path; a GPU is present")
def test_no_device_is_reported(nat):
    p = _params(nat)
    assert nat.lib().nlos_forward(C.byref(p), FAKE, 16, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_ENODEV


def test_python_layer_rejects_cpu_tensors(nat):
    import torch
    import paper_2506_03747_amd as nl
    p = nl.make_params(dict(nx=4, ny=4, half_x=0.5, half_y=0.5), 64, 16.0)
    with pytest.raises(TypeError):
        nl.forward(p, torch.zeros(16, 8))
    with pytest.raises(TypeError):
        nl.patches_from_depth(torch.zeros(4, 4), dict(nx=4, ny=4, half_x=0.5, half_y=0.5))


def test_smooth_and_adjoint_checks(nat):
    """Host-side checks of the smooth forward and the adjoints."""
    L = nat.lib()
    p = _params(nat)
    need = C.c_size_t(0)
    assert L.nlos_forward_smooth_workspace_bytes(C.byref(p), 5000, C.byref(need)) == 0
    assert need.value >= 20 * 32
    assert L.nlos_forward_smooth(C.byref(p), FAKE, 5000, None, FAKE, FAKE, need.value - 1, None) == nat.NLOS_ENOSPC
    nojit = _params(nat, fwhm_ps=0.0)                 # the smooth response needs a jitter width
    assert L.nlos_forward_smooth(C.byref(nojit), FAKE, 16, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_EINVAL
    nc = _params(nat)
    nc.laser = nat.Grid(2, 2, 0.5, 0.5, 0.0, 0.0)      # confocal only
    assert L.nlos_forward_smooth(C.byref(nc), FAKE, 16, None, FAKE, FAKE, 1 << 20, None) == nat.NLOS_EINVAL
    assert L.nlos_adjoint_workspace_bytes(C.byref(nc), 16, C.byref(need)) == nat.NLOS_EINVAL
    assert L.nlos_adjoint_workspace_bytes(C.byref(p), 5000, C.byref(need)) == 0
    assert need.value >= 5000 * 5 * 8                 # fp64 partials per record and scan range
    assert L.nlos_adjoint(C.byref(p), FAKE, 5000, None, FAKE, FAKE, FAKE, need.value - 1, None) == nat.NLOS_ENOSPC
    assert L.nlos_adjoint(C.byref(p), FAKE, 5000, None, None, FAKE, FAKE, need.value, None) == nat.NLOS_EINVAL
    assert L.nlos_adjoint(C.byref(p), FAKE, 5000, None, FAKE, C.c_void_p(0x10004), FAKE, need.value,
                          None) == nat.NLOS_EINVAL
    g = nat.Grid(64, 64, 0.5, 0.5, 0.0, 0.0)
    assert L.nlos_patches_adjoint_workspace_bytes(C.byref(g), C.byref(need)) == 0
    assert need.value == 3 * 4 * 64 * 64
    assert L.nlos_patches_adjoint(C.byref(g), FAKE, None, 1, FAKE, None, FAKE, FAKE, None, FAKE, need.value - 1,
                                  None) == nat.NLOS_ENOSPC
    assert L.nlos_patches_adjoint(C.byref(g), FAKE, None, 3, FAKE, None, FAKE, FAKE, None, FAKE, need.value,
                                  None) == nat.NLOS_EINVAL
    assert L.nlos_patches_adjoint(C.byref(g), None, None, 1, FAKE, None, FAKE, FAKE, None, FAKE, need.value,
                                  None) == nat.NLOS_EINVAL


def test_noise_checks(nat):
    L = nat.lib()
    need = C.c_size_t(0)
    assert L.nlos_noise_scale_workspace_bytes(10**7, C.byref(need)) == 0
    assert need.value == 3 * 8 * 1024
    assert L.nlos_noise_scale_workspace_bytes(-1, C.byref(need)) == nat.NLOS_EINVAL
    assert L.nlos_noise_scale(FAKE, 10**7, 2.0, FAKE, FAKE, need.value - 1, None) == nat.NLOS_ENOSPC
    assert L.nlos_noise_scale(FAKE, 10**7, float("nan"), FAKE, FAKE, need.value, None) == nat.NLOS_EINVAL
    assert L.nlos_noise_scale(FAKE, 10**7, 2.0, C.c_void_p(0x10004), FAKE, need.value, None) == nat.NLOS_EINVAL
    assert L.nlos_poisson_noise(FAKE, 100, None, 1, FAKE, None) == nat.NLOS_EINVAL
    assert L.nlos_poisson_noise(FAKE, -1, FAKE, 1, FAKE, None) == nat.NLOS_EINVAL
    assert L.nlos_poisson_noise(None, 100, FAKE, 1, FAKE, None) == nat.NLOS_EINVAL


def test_lct_checks(nat):
    """Host-side checks of the FFT route (before any device is needed)."""
    L = nat.lib()
    need = C.c_size_t(0)
    p = _params(nat, flags=0, n_bins=64)
    bad = [_params(nat, n_bins=64),                      # cosines requested
           _params(nat, flags=0, n_bins=60),             # not a power of two
           _params(nat, flags=0, n_bins=64, standoff_m=0.5)]
    nc = _params(nat, flags=0, n_bins=64)
    nc.laser = nat.Grid(2, 2, 0.5, 0.5, 0.0, 0.0)
    rect = _params(nat, flags=0, n_bins=64)
    rect.relay.ny = 8
    for q in bad + [nc, rect]:
        assert L.nlos_lct_workspace_bytes(C.byref(q), C.byref(need)) == nat.NLOS_EINVAL
        assert L.nlos_lct_forward(C.byref(q), FAKE, None, None, FAKE, FAKE, 1 << 30, None) == nat.NLOS_EINVAL
    assert L.nlos_lct_forward(C.byref(p), None, None, None, FAKE, FAKE, 1 << 30, None) == nat.NLOS_EINVAL


def test_simulate_checks(nat):
    L = nat.lib()
    p = _params(nat)
    g = nat.Grid(64, 64, 0.5, 0.5, 0.0, 0.0)
    need, geo, fwd = C.c_size_t(0), C.c_size_t(0), C.c_size_t(0)
    assert L.nlos_simulate_workspace_bytes(C.byref(p), C.byref(g), C.byref(need)) == 0
    L.nlos_patches_workspace_bytes(C.byref(g), C.byref(geo))
    L.nlos_forward_workspace_bytes(C.byref(p), 64 * 64, C.byref(fwd))
    assert need.value >= geo.value + fwd.value
    args = (FAKE, None, None, FAKE, FAKE, FAKE)
    assert L.nlos_simulate(C.byref(p), C.byref(g), *args, FAKE, need.value - 1, None, None) == nat.NLOS_ENOSPC
    assert L.nlos_simulate(C.byref(p), C.byref(g), *args, C.c_void_p(0x10010), need.value, None,
                           None) == nat.NLOS_EINVAL
    assert L.nlos_simulate(C.byref(p), C.byref(g), None, None, None, FAKE, FAKE, FAKE, FAKE, need.value, None,
                           None) == nat.NLOS_EINVAL
    bad = _params(nat, bin_ps=0.0)
    assert L.nlos_simulate(C.byref(bad), C.byref(g), *args, FAKE, 1 << 30, None, None) == nat.NLOS_EINVAL
    # a misaligned evaluated-pair counter is rejected before anything is enqueued
    probe = nat.Probe(None, 0x10004)
    assert L.nlos_simulate(C.byref(p), C.byref(g), *args, FAKE, need.value, C.byref(probe), None) == nat.NLOS_EINVAL


def test_tuning_table_and_plan(nat):
    """The tuning table steers the plan; bad entries are rejected."""
    L = nat.lib()
    p = _params(nat, n_bins=1024)
    p.relay.nx = p.relay.ny = 64
    info = nat.PlanInfo()
    assert L.nlos_set_tuning(None, 0) == 0  # the built-in rule
    assert L.nlos_get_plan(C.byref(p), 30000, C.byref(info)) == 0
    default = (info.tl, info.tx, info.ty)
    E = nat.TuningEntry
    for unit in ((1, 2, 2), (1, 4, 4), (1, 2, 1)):
        tab = (E * 1)(E(1, 512, 2048, 1, 1 << 20, *unit))
        assert L.nlos_set_tuning(tab, 1) == 0
        assert L.nlos_get_plan(C.byref(p), 30000, C.byref(info)) == 0
        if unit == (1, 4, 4):
            # 2 x 16 histograms of 1024 u64 bins do not fit in LDS: the rule decides
            assert (info.tl, info.tx, info.ty) == default
        else:
            assert (info.tl, info.tx, info.ty) == unit
    other = (E * 1)(E(1, 1, 100, 1, 1 << 20, 1, 2, 1))      # class that does not match
    assert L.nlos_set_tuning(other, 1) == 0
    L.nlos_get_plan(C.byref(p), 30000, C.byref(info))
    assert (info.tl, info.tx, info.ty) == default
    bad = (E * 1)(E(1, 1, 100, 1, 10, 1, 3, 3))              # unsupported unit
    assert L.nlos_set_tuning(bad, 1) == nat.NLOS_EINVAL
    bad2 = (E * 1)(E(0, 200, 100, 1, 10, 2, 2, 2))           # empty range
    assert L.nlos_set_tuning(bad2, 1) == nat.NLOS_EINVAL
    assert L.nlos_set_tuning(None, 0) == 0
    L.nlos_get_plan(C.byref(p), 30000, C.byref(info))
    assert (info.tl, info.tx, info.ty) == default
    nat._install_tuning(L)                  # the table the package installed at load


def test_tuning_file_is_installed(tmp_path, monkeypatch):
    """tuning.json beside the library is installed when the library loads."""
    import json
    from paper_2506_03747_amd import _native
    tab = tmp_path / "tuning.json"
    tab.write_text(json.dumps({"entries": [dict(confocal=1, t_min=512, t_max=2048, h_min=1, h_max=1 << 20,
                                                tl=1, tx=2, ty=1)]}))
    monkeypatch.setattr(_native, "TUNING_PATH", str(tab))
    monkeypatch.setattr(_native, "_lib", None)
    L = _native.lib()
    try:
        p = _params(_native, n_bins=1024)
        p.relay.nx = p.relay.ny = 64
        info = _native.PlanInfo()
        assert L.nlos_get_plan(C.byref(p), 30000, C.byref(info)) == 0
        assert (info.tl, info.tx, info.ty) == (1, 2, 1)
    finally:
        L.nlos_set_tuning(None, 0)
        _native._install_tuning(L)
    tab.write_text(json.dumps({"entries": [dict(confocal=1, t_min=512, t_max=2048, h_min=1, h_max=9,
                                                tl=1, tx=3, ty=3)]}))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(RuntimeError, match="rejected"):
        _native.lib()
    monkeypatch.setattr(_native, "_lib", None)
    monkeypatch.setenv("NLOS_NO_TUNING", "1")
    _native.lib()
    monkeypatch.delenv("NLOS_NO_TUNING")
    monkeypatch.undo()
    _native.lib().nlos_set_tuning(None, 0)
    _native._install_tuning(_native.lib())
