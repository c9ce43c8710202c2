"""MI355X-native transient NLOS forward operator (arXiv 2506.03747).

Python face of the C ABI in include/nlos.h: PyTorch supplies device memory
and the current HIP stream, the HIP kernels in libnlos.so do every step of
the computation.  Functions take and return torch tensors on the GPU; CPU
tensors are rejected (there is no CPU fallback).

    patches, n_active = patches_from_depth(depth, grid, albedo, mask)
    tau = forward(params, patches, n_active)         # [nx, ny, T] fp32
    tau_s = smooth_transient(depth, albedo, grid, params, mask)   # differentiable

Grids are dicts ``dict(nx, ny, half_x, half_y, cx, cy)`` (metres, cell-centred
on the wall plane z = 0); maps are [nx, ny] (x major).
"""
from __future__ import annotations

import ctypes as C
import json
import os
from typing import Optional

import torch

from ._native import TUNING_PATH  # noqa: F401
from ._native import (NLOS_F_COSINES, NLOS_MAX_BINS, NLOS_MAX_PATCHES, NLOS_MAX_RADIUS,  # noqa: F401
                      NLOS_RECORD_FLOATS, DepthRequest, Grid, NlosError, Params, PlanInfo, Probe, Request,
                      SimRequest, TickCaps, TuningEntry, check, lib, strerror)

__all__ = ["Grid", "Params", "NlosError", "make_grid", "make_params", "params_of",
           "patches_from_depth", "forward", "simulate", "debug_bins", "out_shape", "n_histograms",
           "Batcher", "patches_batched", "forward_batched", "TickGraph", "tick_supported", "forward_smooth",
           "adjoint", "patches_adjoint",
           "SmoothTransient", "smooth_transient", "noise_scale", "poisson_noise", "add_poisson_noise",
           "lct_forward", "set_tuning", "get_plan", "load_tuning", "reset_tuning", "TUNING_PATH"]


def make_grid(g) -> Grid:
    if isinstance(g, Grid):
        return g
    return Grid(int(g["nx"]), int(g["ny"]), float(g["half_x"]), float(g["half_y"]),
                float(g.get("cx", 0.0)), float(g.get("cy", 0.0)))


def make_params(relay, n_bins: int, bin_ps: float, fwhm_ps: float = 0.0, standoff_m: float = 0.0,
                laser=None, cosines: bool = True) -> Params:
    lg = Grid(0, 0, 0.0, 0.0, 0.0, 0.0) if laser is None else make_grid(laser)
    return Params(make_grid(relay), lg, float(standoff_m), float(bin_ps), int(n_bins),
                  NLOS_F_COSINES if cosines else 0, float(fwhm_ps))


def params_of(scene) -> Params:
    """Parameters of any object with relay / laser / n_bins / bin_ps / fwhm_ps /
    standoff_m / cosines attributes."""
    return make_params(scene.relay, scene.n_bins, scene.bin_ps, scene.fwhm_ps, scene.standoff_m,
                       scene.laser, getattr(scene, "cosines", True))


def n_histograms(p: Params) -> int:
    s = p.relay.nx * p.relay.ny
    return s if p.laser.nx == 0 else s * p.laser.nx * p.laser.ny


def out_shape(p: Params):
    if p.laser.nx == 0:
        return (p.relay.nx, p.relay.ny, p.n_bins)
    return (p.laser.nx * p.laser.ny, p.relay.nx, p.relay.ny, p.n_bins)


def _dev(t: Optional[torch.Tensor], dtype, name: str):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a GPU torch tensor (no CPU fallback)")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t: Optional[torch.Tensor]):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream(stream) -> C.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def patches_from_depth(depth: torch.Tensor, grid, albedo: Optional[torch.Tensor] = None,
                       mask: Optional[torch.Tensor] = None, cosines: bool = True,
                       out: Optional[torch.Tensor] = None, n_active: Optional[torch.Tensor] = None,
                       workspace: Optional[torch.Tensor] = None, stream=None):
    """Depth (+ albedo, + mask) maps -> (records [nx*ny, 8] fp32, n_active int32[1])."""
    g = make_grid(grid)
    _dev(depth, torch.float32, "depth")
    _dev(albedo, torch.float32, "albedo")
    _dev(mask, torch.uint8, "mask")
    npx = g.nx * g.ny
    for t, name in ((depth, "depth"), (albedo, "albedo"), (mask, "mask")):
        if t is not None and t.numel() != npx:
            raise ValueError(f"{name} must have {g.nx}x{g.ny} elements")
    dev = depth.device
    if out is None:
        out = torch.empty((npx, NLOS_RECORD_FLOATS), dtype=torch.float32, device=dev)
    if n_active is None:
        n_active = torch.empty(1, dtype=torch.int32, device=dev)
    need = C.c_size_t(0)
    check(lib().nlos_patches_workspace_bytes(C.byref(g), C.byref(need)), "nlos_patches_workspace_bytes")
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(need.value, dtype=torch.uint8, device=dev)
    check(lib().nlos_patches_from_depth(C.byref(g), _ptr(depth), _ptr(albedo), _ptr(mask),
                                        NLOS_F_COSINES if cosines else 0, _ptr(out), _ptr(n_active),
                                        _ptr(workspace), workspace.numel(), _stream(stream)),
          "nlos_patches_from_depth")
    return out, n_active


def forward(params: Params, patches: torch.Tensor, n_active: Optional[torch.Tensor] = None,
            out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Transient histograms, jittered: [nx, ny, T] (confocal) or [L, nx, ny, T]."""
    _dev(patches, torch.float32, "patches")
    _dev(n_active, torch.int32, "n_active")
    if patches.dim() != 2 or patches.shape[1] != NLOS_RECORD_FLOATS:
        raise ValueError("patches must be [n, 8]")
    if out is None:
        out = torch.empty(out_shape(params), dtype=torch.float32, device=patches.device)
    _dev(out, torch.float32, "out")
    if out.numel() != n_histograms(params) * params.n_bins:
        raise ValueError("out has the wrong size")
    need = C.c_size_t(0)
    check(lib().nlos_forward_workspace_bytes(C.byref(params), patches.shape[0], C.byref(need)),
          "nlos_forward_workspace_bytes")
    ws = torch.empty(need.value, dtype=torch.uint8, device=patches.device) if need.value else None
    check(lib().nlos_forward(C.byref(params), _ptr(patches), patches.shape[0], _ptr(n_active), _ptr(out),
                             _ptr(ws), 0 if ws is None else ws.numel(), _stream(stream)),
          "nlos_forward")
    return out


def simulate(params: Params, depth: torch.Tensor, grid, albedo: Optional[torch.Tensor] = None,
             mask: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
             patches: Optional[torch.Tensor] = None, n_active: Optional[torch.Tensor] = None,
             workspace: Optional[torch.Tensor] = None, forward_mark=None, evaluated_pairs=None, stream=None):
    """Depth map -> jittered histograms in one call (geometry, record
    summaries and the forward operator).  Returns (out, patches, n_active).
    ``forward_mark``: a torch.cuda.Event recorded right before the pair
    kernel (timing hook), or None.  ``evaluated_pairs``: a device int64[1]
    the pair kernel adds its evaluated pair count to, or None."""
    g = make_grid(grid)
    _dev(depth, torch.float32, "depth")
    _dev(albedo, torch.float32, "albedo")
    _dev(mask, torch.uint8, "mask")
    npx = g.nx * g.ny
    for t, name in ((depth, "depth"), (albedo, "albedo"), (mask, "mask")):
        if t is not None and t.numel() != npx:
            raise ValueError(f"{name} must have {g.nx}x{g.ny} elements")
    dev = depth.device
    if patches is None:
        patches = torch.empty((npx, NLOS_RECORD_FLOATS), dtype=torch.float32, device=dev)
    if n_active is None:
        n_active = torch.empty(1, dtype=torch.int32, device=dev)
    if out is None:
        out = torch.empty(out_shape(params), dtype=torch.float32, device=dev)
    _dev(out, torch.float32, "out")
    if out.numel() != n_histograms(params) * params.n_bins:
        raise ValueError("out has the wrong size")
    need = C.c_size_t(0)
    check(lib().nlos_simulate_workspace_bytes(C.byref(params), C.byref(g), C.byref(need)),
          "nlos_simulate_workspace_bytes")
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(need.value, dtype=torch.uint8, device=dev)
    probe = None
    if forward_mark is not None or evaluated_pairs is not None:
        _dev(evaluated_pairs, torch.int64, "evaluated_pairs")
        probe = C.byref(Probe(None if forward_mark is None else forward_mark.cuda_event,
                              None if evaluated_pairs is None else evaluated_pairs.data_ptr()))
    check(lib().nlos_simulate(C.byref(params), C.byref(g), _ptr(depth), _ptr(albedo), _ptr(mask), _ptr(patches),
                              _ptr(n_active), _ptr(out), _ptr(workspace), workspace.numel(), probe,
                              _stream(stream)), "nlos_simulate")
    return out, patches, n_active


def debug_bins(params: Params, patches: torch.Tensor, n_active: Optional[torch.Tensor] = None,
               want_u: bool = False, stream=None):
    """Test hook: bin index of every (histogram, record) pair, decided like
    forward(); optionally the fp32 and fp64 arrivals."""
    _dev(patches, torch.float32, "patches")
    _dev(n_active, torch.int32, "n_active")
    H, P = n_histograms(params), patches.shape[0]
    bins = torch.empty((H, P), dtype=torch.int32, device=patches.device)
    uf = ue = None
    if want_u:
        uf = torch.empty((H, P), dtype=torch.float64, device=patches.device)
        ue = torch.empty((H, P), dtype=torch.float64, device=patches.device)
    check(lib().nlos_debug_bins(C.byref(params), _ptr(patches), P, _ptr(n_active), _ptr(bins), _ptr(uf),
                                _ptr(ue), _stream(stream)), "nlos_debug_bins")
    return (bins, uf, ue) if want_u else bins


class Batcher:
    """Reusable buffers of the batched calls: a device workspace per call kind
    that grows as needed, and ``n_tables`` pinned host tables used in turn
    (a table is reused only after an event recorded behind the call that
    last used it has completed), so a loop of batched calls does not block
    on its table uploads."""

    def __init__(self, device="cuda", n_tables: int = 2):
        self.device = torch.device(device)
        self._ws = {}
        self._tables = [None] * max(1, int(n_tables))
        self._events = [None] * len(self._tables)
        self._turn = 0

    def workspace(self, key: str, nbytes: int) -> torch.Tensor:
        ws = self._ws.get(key)
        if ws is None or ws.numel() < nbytes:
            ws = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
            self._ws[key] = ws
        return ws

    def table(self, nbytes: int, stream) -> torch.Tensor:
        i = self._turn
        self._turn = (i + 1) % len(self._tables)
        if self._events[i] is not None:
            self._events[i].synchronize()
        t = self._tables[i]
        if t is None or t.numel() < nbytes:
            t = torch.empty(max(nbytes, 4096), dtype=torch.uint8, pin_memory=True)
            self._tables[i] = t
        self._last = i
        return t

    def mark(self, stream) -> None:
        ev = torch.cuda.Event()
        ev.record(stream)
        self._events[self._last] = ev


def patches_batched(maps, batcher: Optional[Batcher] = None, stream=None):
    """Batched patches_from_depth.  ``maps`` is a list of dicts with keys
    depth, grid and optionally albedo, mask, cosines, out, n_active.
    Returns [(records, n_active)] in the same order."""
    n = len(maps)
    reqs = (DepthRequest * max(n, 1))()
    res = []
    for i, m in enumerate(maps):
        g = make_grid(m["grid"])
        depth = _dev(m["depth"], torch.float32, "depth")
        albedo = _dev(m.get("albedo"), torch.float32, "albedo")
        mask = _dev(m.get("mask"), torch.uint8, "mask")
        npx = g.nx * g.ny
        for t, name in ((depth, "depth"), (albedo, "albedo"), (mask, "mask")):
            if t is not None and t.numel() != npx:
                raise ValueError(f"{name} must have {g.nx}x{g.ny} elements")
        out = m.get("out")
        if out is None:
            out = torch.empty((npx, NLOS_RECORD_FLOATS), dtype=torch.float32, device=depth.device)
        na = m.get("n_active")
        if na is None:
            na = torch.empty(1, dtype=torch.int32, device=depth.device)
        reqs[i] = DepthRequest(g, depth.data_ptr(), None if albedo is None else albedo.data_ptr(),
                               None if mask is None else mask.data_ptr(),
                               NLOS_F_COSINES if m.get("cosines", True) else 0, out.data_ptr(), na.data_ptr())
        res.append((out, na))
    if n == 0:
        return res
    return _run_batched("patches", reqs, n, res, batcher, stream,
                        lib().nlos_patches_batched_sizes, lib().nlos_patches_batched)


def forward_batched(requests, batcher: Optional[Batcher] = None, stream=None):
    """Batched forward.  ``requests`` is a list of (params, patches, n_active,
    out) tuples (n_active and out may be None).  Returns the outputs."""
    n = len(requests)
    reqs = (Request * max(n, 1))()
    outs = []
    for i, (params, patches, n_active, out) in enumerate(requests):
        _dev(patches, torch.float32, "patches")
        _dev(n_active, torch.int32, "n_active")
        if patches.dim() != 2 or patches.shape[1] != NLOS_RECORD_FLOATS:
            raise ValueError("patches must be [n, 8]")
        if out is None:
            out = torch.empty(out_shape(params), dtype=torch.float32, device=patches.device)
        _dev(out, torch.float32, "out")
        if out.numel() != n_histograms(params) * params.n_bins:
            raise ValueError("out has the wrong size")
        reqs[i] = Request(params, patches.data_ptr(), patches.shape[0],
                          None if n_active is None else n_active.data_ptr(), out.data_ptr())
        outs.append(out)
    if n == 0:
        return outs
    return _run_batched("forward", reqs, n, outs, batcher, stream,
                        lib().nlos_forward_batched_sizes, lib().nlos_forward_batched)


def _run_batched(key, reqs, n, result, batcher, stream, sizes_fn, run_fn):
    tb, wb = C.c_size_t(0), C.c_size_t(0)
    check(sizes_fn(reqs, n, C.byref(tb), C.byref(wb)), f"{key} batched sizes")
    st = torch.cuda.current_stream() if stream is None else stream
    if batcher is None:
        ws = torch.empty(max(wb.value, 256), dtype=torch.uint8, device="cuda")
        table = None
        tptr, tlen = None, 0
    else:
        ws = batcher.workspace(key, wb.value)
        table = batcher.table(tb.value, st)
        tptr, tlen = C.c_void_p(table.data_ptr()), table.numel()
    check(run_fn(reqs, n, tptr, tlen, _ptr(ws), ws.numel(), C.c_void_p(st.cuda_stream)), f"{key} batched")
    if batcher is not None:
        batcher.mark(st)
    return result


def tick_supported(params: Params, grid) -> bool:
    """Whether a request can run in a serving tick: confocal, a map of at most
    4096 enumeration blocks of 256 pixels, and a plan that pairs units over the
    whole window."""
    g = make_grid(grid)
    if params.laser.nx != 0 or params.laser.ny != 0:
        return False
    if -(-g.nx // 16) * -(-g.ny // 16) * 256 > 4096 * 256:
        return False
    plan = get_plan(params, g.nx * g.ny)
    return plan["pair"] == 1 and plan["n_windows"] == 1


class TickGraph:
    """One serving-tick slot: a pinned host table, a device workspace and the
    library's tick graph over them (instantiated once).  Per tick:
    ``plan(requests)`` writes the table, ``launch(stream)`` launches the
    graph (one launch; the pair node's grid follows the tick).  A slot holds
    one tick at a time: plan the next only once the previous launch has
    passed (``event`` is recorded behind each launch).

    requests: dicts with params, grid, depth, albedo, mask and, optionally,
    out, patches, n_active (allocated here on the current stream if absent).
    ``graph=False`` launches the same four operations without the graph."""

    def __init__(self, max_requests: int, max_pixels: int, device="cuda", graph: bool = True):
        self.device = torch.device(device)
        self.caps = TickCaps(int(max_requests), int(max_pixels))
        tb, wb = C.c_size_t(0), C.c_size_t(0)
        check(lib().nlos_tick_sizes(C.byref(self.caps), C.byref(tb), C.byref(wb)), "nlos_tick_sizes")
        self.table = torch.empty(tb.value, dtype=torch.uint8, pin_memory=True)
        self.ws = torch.empty(wb.value, dtype=torch.uint8, device=self.device)
        self.event = None
        self._handle = None
        self._lib = lib()
        if graph:
            h = C.c_void_p()
            check(self._lib.nlos_tick_graph_create(C.byref(self.caps), _ptr(self.table), _ptr(self.ws),
                                                   self.ws.numel(), C.byref(h)), "nlos_tick_graph_create")
            self._handle = h

    @property
    def bytes(self) -> int:
        return self.ws.numel()

    def busy(self) -> bool:
        return self.event is not None and not self.event.query()

    def plan(self, requests):
        """Write the tick table for ``requests``; returns [(out, patches, n_active)]."""
        n = len(requests)
        arr = (SimRequest * max(n, 1))()
        res = []
        for i, r in enumerate(requests):
            prm, g = r["params"], make_grid(r["grid"])
            depth = _dev(r["depth"], torch.float32, "depth")
            albedo = _dev(r.get("albedo"), torch.float32, "albedo")
            mask = _dev(r.get("mask"), torch.uint8, "mask")
            npx = g.nx * g.ny
            for t, name in ((depth, "depth"), (albedo, "albedo"), (mask, "mask")):
                if t is not None and t.numel() != npx:
                    raise ValueError(f"{name} must have {g.nx}x{g.ny} elements")
            out = r.get("out")
            if out is None:
                out = torch.empty(out_shape(prm), dtype=torch.float32, device=self.device)
            patches = r.get("patches")
            if patches is None:
                patches = torch.empty((npx, NLOS_RECORD_FLOATS), dtype=torch.float32, device=self.device)
            na = r.get("n_active")
            if na is None:
                na = torch.empty(1, dtype=torch.int32, device=self.device)
            _dev(out, torch.float32, "out")
            if out.numel() != n_histograms(prm) * prm.n_bins:
                raise ValueError("out has the wrong size")
            arr[i] = SimRequest(prm, g, depth.data_ptr(), None if albedo is None else albedo.data_ptr(),
                                None if mask is None else mask.data_ptr(), patches.data_ptr(), na.data_ptr(),
                                out.data_ptr())
            res.append((out, patches, na))
        if self.busy():
            raise RuntimeError("tick slot still in flight")
        check(self._lib.nlos_tick_plan(C.byref(self.caps), arr, n, _ptr(self.table), self.table.numel(),
                                       _ptr(self.ws), self.ws.numel()), "nlos_tick_plan")
        return res

    def launch(self, stream=None):
        st = torch.cuda.current_stream(self.device) if stream is None else stream
        if self._handle is not None:
            check(self._lib.nlos_tick_graph_launch(self._handle, C.c_void_p(st.cuda_stream)), "nlos_tick_graph_launch")
        else:
            check(self._lib.nlos_tick_launch(C.byref(self.caps), _ptr(self.table), _ptr(self.ws), self.ws.numel(),
                                             C.c_void_p(st.cuda_stream)), "nlos_tick_launch")
        self.event = torch.cuda.Event()
        self.event.record(st)
        return self.event

    def close(self):
        if self._handle is not None:
            if self.event is not None:
                self.event.synchronize()
            self._lib.nlos_tick_graph_destroy(self._handle)
            self._handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001 - interpreter shutdown
            pass


def _ws(nbytes: int, device):
    return torch.empty(max(int(nbytes), 16), dtype=torch.uint8, device=device)


def forward_smooth(params: Params, patches: torch.Tensor, n_active: Optional[torch.Tensor] = None,
                   out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Smooth-response histograms (continuous Gaussian per pair), confocal
    [nx, ny, T]."""
    _dev(patches, torch.float32, "patches")
    _dev(n_active, torch.int32, "n_active")
    if patches.dim() != 2 or patches.shape[1] != NLOS_RECORD_FLOATS:
        raise ValueError("patches must be [n, 8]")
    if out is None:
        out = torch.empty(out_shape(params), dtype=torch.float32, device=patches.device)
    _dev(out, torch.float32, "out")
    if out.numel() != n_histograms(params) * params.n_bins:
        raise ValueError("out has the wrong size")
    need = C.c_size_t(0)
    check(lib().nlos_forward_smooth_workspace_bytes(C.byref(params), patches.shape[0], C.byref(need)),
          "nlos_forward_smooth_workspace_bytes")
    ws = _ws(need.value, patches.device)
    check(lib().nlos_forward_smooth(C.byref(params), _ptr(patches), patches.shape[0], _ptr(n_active), _ptr(out),
                                    _ptr(ws), ws.numel(), _stream(stream)), "nlos_forward_smooth")
    return out


def adjoint(params: Params, patches: torch.Tensor, n_active: Optional[torch.Tensor], grad_out: torch.Tensor,
            out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Record gradients [n, 8] ({0, 0, dz, da, dn_x, dn_y, dn_z, 0}) of the
    smooth forward for the upstream gradient ``grad_out`` [nx, ny, T]."""
    _dev(patches, torch.float32, "patches")
    _dev(n_active, torch.int32, "n_active")
    _dev(grad_out, torch.float32, "grad_out")
    if grad_out.numel() != n_histograms(params) * params.n_bins:
        raise ValueError("grad_out has the wrong size")
    if out is None:
        out = torch.empty((patches.shape[0], NLOS_RECORD_FLOATS), dtype=torch.float32, device=patches.device)
    _dev(out, torch.float32, "out")
    need = C.c_size_t(0)
    check(lib().nlos_adjoint_workspace_bytes(C.byref(params), patches.shape[0], C.byref(need)),
          "nlos_adjoint_workspace_bytes")
    ws = _ws(need.value, patches.device)
    check(lib().nlos_adjoint(C.byref(params), _ptr(patches), patches.shape[0], _ptr(n_active), _ptr(grad_out),
                             _ptr(out), _ptr(ws), ws.numel(), _stream(stream)), "nlos_adjoint")
    return out


def patches_adjoint(grid, depth: torch.Tensor, albedo: Optional[torch.Tensor], patches: torch.Tensor,
                    n_active: Optional[torch.Tensor], grad_rec: torch.Tensor, cosines: bool = True,
                    want_albedo: bool = True, stream=None):
    """Record gradients -> (grad_depth [nx, ny], grad_albedo [nx, ny] or None)."""
    g = make_grid(grid)
    _dev(depth, torch.float32, "depth")
    _dev(albedo, torch.float32, "albedo")
    _dev(patches, torch.float32, "patches")
    _dev(n_active, torch.int32, "n_active")
    _dev(grad_rec, torch.float32, "grad_rec")
    npx = g.nx * g.ny
    if depth.numel() != npx or patches.shape[0] != npx or grad_rec.shape[0] != npx:
        raise ValueError("maps, records and record gradients must cover the grid")
    gd = torch.empty((g.nx, g.ny), dtype=torch.float32, device=depth.device)
    ga = torch.empty((g.nx, g.ny), dtype=torch.float32, device=depth.device) if want_albedo else None
    need = C.c_size_t(0)
    check(lib().nlos_patches_adjoint_workspace_bytes(C.byref(g), C.byref(need)),
          "nlos_patches_adjoint_workspace_bytes")
    ws = _ws(need.value, depth.device)
    check(lib().nlos_patches_adjoint(C.byref(g), _ptr(depth), _ptr(albedo), NLOS_F_COSINES if cosines else 0,
                                     _ptr(patches), _ptr(n_active), _ptr(grad_rec), _ptr(gd), _ptr(ga), _ptr(ws),
                                     ws.numel(), _stream(stream)), "nlos_patches_adjoint")
    return gd, ga


class SmoothTransient(torch.autograd.Function):
    """tau_s = smooth forward of the depth (and albedo) maps; backward by the
    hand-written adjoint kernels (record gradients, then the depth stencil)."""

    @staticmethod
    def forward(ctx, depth, albedo, grid, params, mask):
        cos = bool(params.flags & NLOS_F_COSINES)
        depth = depth.contiguous()
        albedo = None if albedo is None else albedo.contiguous()
        rec, n = patches_from_depth(depth, grid, albedo, mask, cosines=cos)
        tau = forward_smooth(params, rec, n)
        ctx.grid, ctx.params, ctx.cos = grid, params, cos
        ctx.has_albedo = albedo is not None
        ctx.save_for_backward(depth, albedo if albedo is not None else depth, rec, n)
        return tau

    @staticmethod
    def backward(ctx, grad_tau):
        depth, albedo, rec, n = ctx.saved_tensors
        if not ctx.has_albedo:
            albedo = None
        grad_rec = adjoint(ctx.params, rec, n, grad_tau.contiguous())
        gd, ga = patches_adjoint(ctx.grid, depth, albedo, rec, n, grad_rec, cosines=ctx.cos,
                                 want_albedo=ctx.has_albedo and ctx.needs_input_grad[1])
        return gd, ga, None, None, None


def smooth_transient(depth: torch.Tensor, albedo: Optional[torch.Tensor], grid, params: Params,
                     mask: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Differentiable smooth forward of depth and albedo maps (confocal)."""
    return SmoothTransient.apply(depth, albedo, grid, params, mask)


def noise_scale(tau: torch.Tensor, nr_db: float, stream=None) -> torch.Tensor:
    """Device double[3] {mean, population variance, sigma_n = Var / 10^(nr/10)}
    of a whole frame."""
    _dev(tau, torch.float32, "tau")
    n = tau.numel()
    need = C.c_size_t(0)
    check(lib().nlos_noise_scale_workspace_bytes(n, C.byref(need)), "nlos_noise_scale_workspace_bytes")
    ws = _ws(need.value, tau.device)
    stats = torch.empty(3, dtype=torch.float64, device=tau.device)
    check(lib().nlos_noise_scale(_ptr(tau), n, float(nr_db), _ptr(stats), _ptr(ws), ws.numel(), _stream(stream)),
          "nlos_noise_scale")
    return stats


def poisson_noise(tau: torch.Tensor, sigma_n: torch.Tensor, seed: int, out: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Poisson(tau * s) / s elementwise, s = sigma_n[0] (device double)."""
    _dev(tau, torch.float32, "tau")
    _dev(sigma_n, torch.float64, "sigma_n")
    if out is None:
        out = torch.empty_like(tau)
    _dev(out, torch.float32, "out")
    if out.numel() != tau.numel():
        raise ValueError("out has the wrong size")
    check(lib().nlos_poisson_noise(_ptr(tau), tau.numel(), _ptr(sigma_n), C.c_uint64(int(seed) & (2**64 - 1)),
                                   _ptr(out), _stream(stream)), "nlos_poisson_noise")
    return out


def add_poisson_noise(tau: torch.Tensor, nr_db: float, seed: int, out: Optional[torch.Tensor] = None,
                      stream=None) -> torch.Tensor:
    """Algorithm 1 step 2.4 on a (jittered) frame: sigma_n from the frame's
    variance, then Poisson(tau sigma_n) / sigma_n; no host synchronisation."""
    stats = noise_scale(tau, nr_db, stream)
    return poisson_noise(tau, stats[2:], seed, out=out, stream=stream)


def lct_forward(params: Params, depth: torch.Tensor, albedo: Optional[torch.Tensor] = None,
                mask: Optional[torch.Tensor] = None, out: Optional[torch.Tensor] = None,
                workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The paper's FFT (light-cone) forward route, [N, N, M] fp32: confocal
    N x N scan co-registered with the N x N depth map, no stand-off, no
    cosines (params.flags = 0), M a power of two."""
    _dev(depth, torch.float32, "depth")
    _dev(albedo, torch.float32, "albedo")
    _dev(mask, torch.uint8, "mask")
    n = params.relay.nx
    for t, name in ((depth, "depth"), (albedo, "albedo"), (mask, "mask")):
        if t is not None and t.numel() != n * params.relay.ny:
            raise ValueError(f"{name} must cover the scan grid")
    if out is None:
        out = torch.empty(out_shape(params), dtype=torch.float32, device=depth.device)
    _dev(out, torch.float32, "out")
    need = C.c_size_t(0)
    check(lib().nlos_lct_workspace_bytes(C.byref(params), C.byref(need)), "nlos_lct_workspace_bytes")
    if workspace is None or workspace.numel() < need.value:
        workspace = torch.empty(need.value, dtype=torch.uint8, device=depth.device)
    check(lib().nlos_lct_forward(C.byref(params), _ptr(depth), _ptr(albedo), _ptr(mask), _ptr(out), _ptr(workspace),
                                 workspace.numel(), _stream(stream)), "nlos_lct_forward")
    return out


def set_tuning(entries) -> None:
    """Install a tuning table: a list of dicts with confocal, t_min, t_max,
    h_min, h_max, tl, tx, ty (an empty list clears it)."""
    n = len(entries)
    arr = (TuningEntry * max(n, 1))()
    for i, e in enumerate(entries):
        arr[i] = TuningEntry(int(e["confocal"]), int(e["t_min"]), int(e["t_max"]), int(e["h_min"]),
                             int(e["h_max"]), int(e["tl"]), int(e["tx"]), int(e["ty"]))
    check(lib().nlos_set_tuning(arr, n), "nlos_set_tuning")


def get_plan(params: Params, n_patches: int) -> dict:
    """The launch plan nlos_forward would use (unit, pairing, split, windows)."""
    info = PlanInfo()
    check(lib().nlos_get_plan(C.byref(params), int(n_patches), C.byref(info)), "nlos_get_plan")
    return {k: getattr(info, k) for k, _ in PlanInfo._fields_}


def load_tuning(path: str = TUNING_PATH) -> bool:
    """Install the table written by the autotuner, if there is one."""
    if not os.path.exists(path):
        return False
    with open(path) as f:
        set_tuning(json.load(f)["entries"])
    return True


def reset_tuning() -> None:
    """Back to the table installed at load: tuning.json if present (and
    NLOS_NO_TUNING unset), else none."""
    set_tuning([])
    if not os.environ.get("NLOS_NO_TUNING"):
        load_tuning()
