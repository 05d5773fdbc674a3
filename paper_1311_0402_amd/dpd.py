"""Python binding of libdpd with torch tensors as device memory.

The functions named like the C entry points (``dpd_bin_reorder``,
``dpd_build_neighbors``, ``dpd_forces``, ``dpd_step``,
``dpd_forces_backward``) only marshal arguments: every step of the method
runs in the HIP kernels behind include/dpd.h.  ``System`` owns the device
buffers one simulation needs and strings the calls together.
"""
from __future__ import annotations

import ctypes as C
import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np
import torch

from . import _abi
from ._abi import DPDError, check, lib

FP64 = _abi.FP64
MIXED = _abi.MIXED


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("libdpd takes device tensors only")
    if not t.is_contiguous():
        raise ValueError("libdpd takes contiguous tensors only")
    return t.data_ptr()


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


@dataclass
class Params:
    """Physical and numerical parameters (mirrors dpd_params)."""

    box: tuple
    r_c: float = 1.0
    skin: float = 0.0
    dt: float = 0.01
    lam: float = 0.5
    s: float = 0.5
    n_types: int = 1
    a: np.ndarray = field(default_factory=lambda: np.array([[25.0]]))
    gamma: np.ndarray = field(default_factory=lambda: np.array([[4.5]]))
    sigma: np.ndarray = field(default_factory=lambda: np.array([[3.0]]))
    seed: int = 0
    body_g: float = 0.0
    body_split: float = 0.0
    bond_k: float = 0.0
    bond_r0: float = 0.0
    partner: Optional[torch.Tensor] = None      # device int32 [n, 2] by tag

    @classmethod
    def like(cls, obj, device="cuda", skin: float = 0.0) -> "Params":
        """Parameters copied from any object with the same attribute names."""
        partner = getattr(obj, "partner", None)
        if partner is not None and not isinstance(partner, torch.Tensor):
            partner = torch.as_tensor(np.ascontiguousarray(partner, dtype=np.int32), device=device)
        return cls(box=tuple(float(b) for b in obj.box), r_c=float(obj.r_c), skin=skin,
                   dt=float(obj.dt), lam=float(obj.lam), s=float(obj.s), n_types=int(obj.n_types),
                   a=np.asarray(obj.a, dtype=np.float64), gamma=np.asarray(obj.gamma, dtype=np.float64),
                   sigma=np.asarray(obj.sigma, dtype=np.float64), seed=int(obj.seed),
                   body_g=float(obj.body_g), body_split=float(obj.body_split),
                   bond_k=float(obj.bond_k), bond_r0=float(obj.bond_r0), partner=partner)

    def c(self) -> _abi.dpd_params:
        p = _abi.dpd_params()
        for k in range(3):
            p.box[k] = float(self.box[k])
        p.r_c, p.skin, p.dt, p.lam, p.s = self.r_c, self.skin, self.dt, self.lam, self.s
        nt = int(self.n_types)
        p.n_types = nt
        for name in ("a", "gamma", "sigma"):
            if not 1 <= nt <= _abi.MAX_TYPES:
                break                     # the library rejects n_types itself
            tab = np.asarray(getattr(self, name), dtype=np.float64).reshape(-1)
            if tab.size != nt * nt:
                raise ValueError(f"{name} must have n_types^2 entries")
            arr = getattr(p, name)
            for t in range(nt * nt):
                arr[t] = float(tab[t])
        p.seed = int(self.seed) & ((1 << 64) - 1)
        p.body_g, p.body_split = self.body_g, self.body_split
        p.bond_k, p.bond_r0 = self.bond_k, self.bond_r0
        p.bond_partner = _ptr(self.partner) if self.partner is not None else None
        return p

    @property
    def r_list(self) -> float:
        return self.r_c + self.skin


@dataclass
class State:
    x: torch.Tensor        # float64 [3, n]
    v: torch.Tensor        # float64 [3, n]
    f: torch.Tensor        # float64 [3, n]
    tag: torch.Tensor      # int32 [n] (read as uint32)
    type: torch.Tensor     # uint8 [n]

    @property
    def n(self) -> int:
        return int(self.x.shape[1])

    @classmethod
    def empty(cls, n: int, device="cuda") -> "State":
        return cls(x=torch.empty((3, n), dtype=torch.float64, device=device),
                   v=torch.empty((3, n), dtype=torch.float64, device=device),
                   f=torch.zeros((3, n), dtype=torch.float64, device=device),
                   tag=torch.empty(n, dtype=torch.int32, device=device),
                   type=torch.empty(n, dtype=torch.uint8, device=device))

    def c(self) -> _abi.dpd_state:
        s = _abi.dpd_state()
        s.n = self.n
        s.x, s.v, s.f = _ptr(self.x), _ptr(self.v), _ptr(self.f)
        s.tag, s.type = _ptr(self.tag), _ptr(self.type)
        return s


@dataclass
class Cells:
    cell_start: torch.Tensor   # int32 [n_cells + 1]
    cell_xyz: torch.Tensor     # int32 [n] (packed cx | cy<<10 | cz<<20)
    perm: torch.Tensor         # int32 [n]
    idx_of_tag: torch.Tensor   # int32 [n]

    @classmethod
    def empty(cls, n: int, n_cells: int, device="cuda") -> "Cells":
        i32 = dict(dtype=torch.int32, device=device)
        return cls(torch.empty(n_cells + 1, **i32), torch.empty(max(n, 1), **i32),
                   torch.empty(max(n, 1), **i32), torch.full((max(n, 1),), -1, **i32))

    def c(self) -> _abi.dpd_cells:
        c = _abi.dpd_cells()
        c.cell_start, c.cell_xyz = _ptr(self.cell_start), _ptr(self.cell_xyz)
        c.perm, c.idx_of_tag = _ptr(self.perm), _ptr(self.idx_of_tag)
        return c


@dataclass
class NList:
    offset: torch.Tensor       # int32 [n + 1]
    index: torch.Tensor        # int32 [capacity]

    @property
    def capacity(self) -> int:
        return int(self.index.numel())

    @classmethod
    def empty(cls, n: int, capacity: int, device="cuda") -> "NList":
        return cls(torch.zeros(n + 1, dtype=torch.int32, device=device),
                   torch.empty(max(int(capacity), 1), dtype=torch.int32, device=device))

    def c(self) -> _abi.dpd_nlist:
        c = _abi.dpd_nlist()
        c.capacity = self.capacity
        c.offset, c.index = _ptr(self.offset), _ptr(self.index)
        return c


# ----------------------------------------------------------------- queries --

def cell_grid(params: Params):
    nc = (C.c_int32 * 3)()
    check(lib().dpd_cell_grid(C.byref(params.c()), nc), "dpd_cell_grid")
    return tuple(int(v) for v in nc)


def set_pair_evaluation(mode: int) -> int:
    """0: every list entry is evaluated; 1: a pair inside one 64-particle
    chunk is evaluated once; 2 (default): once in the FP64 form, every entry
    in the mixed form.  Returns the previous mode."""
    rc = lib().dpd_set_pair_evaluation(int(mode))
    if rc < 0:
        check(rc, "dpd_set_pair_evaluation")
    return int(rc)


def set_list_builder(kind: int) -> int:
    """The neighbour-list builder of single-system calls: 0 (default) tile
    builder, 1 wave per 2x2x2-cell block, 2 lane per particle; all write the
    same rows.  Returns the previous kind."""
    rc = lib().dpd_set_list_builder(int(kind))
    if rc < 0:
        check(rc, "dpd_set_list_builder")
    return int(rc)


def workspace_bytes(params: Params, n: int, precision: int = FP64) -> int:
    nb = lib().dpd_workspace_bytes(C.byref(params.c()), int(n), int(precision))
    if nb == 0:
        raise DPDError(_abi.DPD_EINVAL, "dpd_workspace_bytes")
    return int(nb)


def alloc_workspace(params: Params, n: int, precision: int = FP64, device="cuda") -> torch.Tensor:
    nb = workspace_bytes(params, n, precision)
    # torch's caching allocator hands out 512-byte aligned blocks
    return torch.empty(nb, dtype=torch.uint8, device=device)


def default_capacity(params: Params, n: int, slack: float = 1.5) -> int:
    vol = float(np.prod(params.box))
    mean = 4.0 / 3.0 * math.pi * (n / vol) * params.r_list ** 3
    return int(slack * n * mean) + 4096


# -------------------------------------------------- entry points (marshal) --

def dpd_bin_reorder(params: Params, src: State, dst: State, cells: Cells, ws: torch.Tensor,
                    x32=None, v32=None, stream=None) -> None:
    s_in, s_out, c = src.c(), dst.c(), cells.c()
    check(lib().dpd_bin_reorder(C.byref(params.c()), C.byref(s_in), C.byref(s_out), C.byref(c),
                                _ptr(x32), _ptr(v32), _ptr(ws), ws.numel(), _stream(stream)),
          "dpd_bin_reorder")


def dpd_build_neighbors(params: Params, st: State, cells: Cells, x32: torch.Tensor, nl: NList,
                        status: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    s, c, n = st.c(), cells.c(), nl.c()
    check(lib().dpd_build_neighbors(C.byref(params.c()), C.byref(s), C.byref(c), _ptr(x32), C.byref(n),
                                    _ptr(status), _ptr(ws), ws.numel(), _stream(stream)),
          "dpd_build_neighbors")


def dpd_forces(params: Params, precision: int, st: State, cells: Optional[Cells], nl: NList, step: int,
               f_out: torch.Tensor, ws: torch.Tensor, *, x32=None, v32=None, pe_out=None, stats=None,
               status=None, stream=None) -> None:
    s, n = st.c(), nl.c()
    c = cells.c() if cells is not None else None
    check(lib().dpd_forces(C.byref(params.c()), int(precision), C.byref(s),
                           C.byref(c) if c is not None else None, _ptr(x32), _ptr(v32), C.byref(n),
                           int(step), _ptr(f_out), _ptr(pe_out), _ptr(stats), _ptr(status),
                           _ptr(ws), ws.numel(), _stream(stream)),
          "dpd_forces")


def dpd_forces_noalloc(params: Params, precision: int, st: State, cells: Optional[Cells], nl: NList, step: int,
                       f_out: torch.Tensor, *, x32=None, v32=None, pe_out=None, stats=None, status=None,
                       stream=None) -> None:
    s, n = st.c(), nl.c()
    c = cells.c() if cells is not None else None
    check(lib().dpd_forces_noalloc(C.byref(params.c()), int(precision), C.byref(s),
                                   C.byref(c) if c is not None else None, _ptr(x32), _ptr(v32), C.byref(n),
                                   int(step), _ptr(f_out), _ptr(pe_out), _ptr(stats), _ptr(status),
                                   _stream(stream)),
          "dpd_forces_noalloc")


def dpd_step(params: Params, precision: int, st: State, n_steps: int, d_step: torch.Tensor,
             cells: Cells, nl: NList, status: torch.Tensor, ws: torch.Tensor, *, reductions=None,
             x32=None, v32=None, phase_events=None, stream=None) -> None:
    """phase_events: optional list of 6 * n_steps recorded torch.cuda.Events."""
    s, c, n = st.c(), cells.c(), nl.c()
    ev = None
    if phase_events is not None:
        if len(phase_events) != 6 * n_steps:
            raise ValueError("phase_events needs 6 events per step")
        handles = [e.cuda_event for e in phase_events]
        if not all(handles):
            raise ValueError("record every event once before passing it (torch creates them lazily)")
        ev = (C.c_void_p * len(handles))(*handles)
    check(lib().dpd_step(C.byref(params.c()), int(precision), C.byref(s), int(n_steps), _ptr(d_step),
                         _ptr(reductions), C.byref(c), C.byref(n), _ptr(x32), _ptr(v32), _ptr(status),
                         ev, _ptr(ws), ws.numel(), _stream(stream)),
          "dpd_step")


def dpd_forces_backward(params: Params, st: State, cells: Optional[Cells], nl: NList, step: int,
                        grad_f: torch.Tensor, grad_x: torch.Tensor, grad_v: torch.Tensor,
                        grad_a: torch.Tensor, grad_gamma: torch.Tensor, ws: torch.Tensor,
                        accumulate: bool = False, stream=None) -> None:
    s, n = st.c(), nl.c()
    c = cells.c() if cells is not None else None
    check(lib().dpd_forces_backward(C.byref(params.c()), C.byref(s), C.byref(c) if c is not None else None,
                                    C.byref(n), int(step), _ptr(grad_f), _ptr(grad_x), _ptr(grad_v),
                                    _ptr(grad_a), _ptr(grad_gamma), 1 if accumulate else 0, _ptr(ws),
                                    ws.numel(), _stream(stream)),
          "dpd_forces_backward")


def dpd_step_backward(params: Params, st: State, cells: Cells, nl: NList, step: int,
                      gx_in: torch.Tensor, gv_in: torch.Tensor, gf_in: torch.Tensor,
                      gx_out: torch.Tensor, gv_out: torch.Tensor, gf_out: torch.Tensor,
                      grad_a: torch.Tensor, grad_gamma: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    s, c, n = st.c(), cells.c(), nl.c()
    check(lib().dpd_step_backward(C.byref(params.c()), C.byref(s), C.byref(c), C.byref(n), int(step),
                                  _ptr(gx_in), _ptr(gv_in), _ptr(gf_in), _ptr(gx_out), _ptr(gv_out),
                                  _ptr(gf_out), _ptr(grad_a), _ptr(grad_gamma), _ptr(ws), ws.numel(),
                                  _stream(stream)),
          "dpd_step_backward")


# ------------------------------------------------- border exchange (Alg 6) --

def border_workspace(n: int, device="cuda") -> torch.Tensor:
    nb = lib().dpd_border_workspace_bytes(int(n))
    if nb == 0:
        raise DPDError(_abi.DPD_EINVAL, "dpd_border_workspace_bytes")
    return torch.empty(int(nb), dtype=torch.uint8, device=device)


def ghost_records(capacity: int, device="cuda") -> torch.Tensor:
    """Device buffer of `capacity` dpd_ghost records (56 bytes each), as
    float64 words [capacity, 7]: x, y, z, vx, vy, vz, (tag, type) bits."""
    assert _abi.GHOST_BYTES == 56
    return torch.empty((max(int(capacity), 1), 7), dtype=torch.float64, device=device)


def dpd_border_lists(st: State, lo, hi, width: float, face_mask: int, send_offset: torch.Tensor,
                     send_index: torch.Tensor, status: torch.Tensor, ws: torch.Tensor, stream=None) -> None:
    s = st.c()
    lo_c = (C.c_double * 3)(*[float(v) for v in lo])
    hi_c = (C.c_double * 3)(*[float(v) for v in hi])
    check(lib().dpd_border_lists(C.byref(s), lo_c, hi_c, float(width), int(face_mask), _ptr(send_offset),
                                 _ptr(send_index), int(send_index.numel()), _ptr(status), _ptr(ws), ws.numel(),
                                 _stream(stream)), "dpd_border_lists")


def dpd_border_pack(st: State, send_offset: torch.Tensor, send_index: torch.Tensor, shift, records: torch.Tensor,
                    status: torch.Tensor, stream=None) -> None:
    s = st.c()
    sh = np.ascontiguousarray(shift, dtype=np.float64).reshape(18)
    sh_c = (C.c_double * 18)(*[float(v) for v in sh])
    cap = min(int(send_index.numel()), int(records.shape[0]))
    check(lib().dpd_border_pack(C.byref(s), _ptr(send_offset), _ptr(send_index), cap, sh_c, _ptr(records),
                                _ptr(status), _stream(stream)), "dpd_border_pack")


def dpd_border_unpack(records: torch.Tensor, d_count: torch.Tensor, dst: State, first: int, status: torch.Tensor,
                      stream=None) -> None:
    s = dst.c()
    check(lib().dpd_border_unpack(_ptr(records), _ptr(d_count), int(records.shape[0]), C.byref(s), int(first),
                                  _ptr(status), _stream(stream)), "dpd_border_unpack")


# ------------------------------------- the paper's numerics (A/B study) --

def math_eval(fn: int, a: torch.Tensor, b: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    out = torch.empty_like(a)
    check(lib().dpd_math_eval(int(fn), int(a.numel()), _ptr(a), _ptr(b), _ptr(out), _stream(stream)),
          "dpd_math_eval")
    return out


def math_latency(fn: int, chain: int, stream=None) -> int:
    """Shader-clock ticks of one wave's chain of `chain` dependent calls (synchronises)."""
    cyc = torch.zeros(1, dtype=torch.int64, device="cuda")
    sink = torch.empty(64, dtype=torch.float64, device="cuda")
    check(lib().dpd_math_latency(int(fn), int(chain), _ptr(cyc), _ptr(sink), _stream(stream)), "dpd_math_latency")
    return int(cyc.item())


def tea_signatures(tag: torch.Tensor, v: torch.Tensor, step: int, seed: int, stream=None) -> torch.Tensor:
    n = int(tag.numel())
    sig = torch.empty(max(n, 1), dtype=torch.int32, device=tag.device)
    check(lib().dpd_tea_signatures(n, _ptr(tag), _ptr(v), int(step), int(seed) & ((1 << 64) - 1), _ptr(sig),
                                   _stream(stream)), "dpd_tea_signatures")
    return sig[:n]


def tea_gaussians(sig_i: torch.Tensor, sig_j: torch.Tensor, step: int, seed: int, stream=None):
    n = int(sig_i.numel())
    words = torch.empty((max(n, 1), 2), dtype=torch.int32, device=sig_i.device)
    xi = torch.empty(max(n, 1), dtype=torch.float64, device=sig_i.device)
    check(lib().dpd_tea_gaussians(n, _ptr(sig_i), _ptr(sig_j), int(step), int(seed) & ((1 << 64) - 1),
                                  _ptr(words), _ptr(xi), _stream(stream)), "dpd_tea_gaussians")
    return words[:n], xi[:n]


def gaussian_throughput(generator: int, n_tags: int, pairs_per_thread: int, step: int, seed: int,
                        sig: Optional[torch.Tensor], sink: torch.Tensor, stream=None) -> None:
    check(lib().dpd_gaussian_throughput(int(generator), int(n_tags), int(pairs_per_thread), int(step),
                                        int(seed) & ((1 << 64) - 1), _ptr(sig), _ptr(sink), _stream(stream)),
          "dpd_gaussian_throughput")


# ------------------------------------------------------------------ System --

class System:
    """Device buffers of one DPD system plus the per-step driver.

    After ``load`` the state is reordered, its neighbour list built and the
    forces of the current step computed, so ``step`` can run immediately.
    """

    def __init__(self, params: Params, n: int, precision: int = FP64, capacity: Optional[int] = None,
                 device="cuda"):
        self.params = params
        self.n = int(n)
        self.precision = int(precision)
        self.device = device
        self.nc = cell_grid(params)
        n_cells = self.nc[0] * self.nc[1] * self.nc[2]
        self.state = State.empty(self.n, device)
        self.cells = Cells.empty(self.n, n_cells, device)
        self.nlist = NList.empty(self.n, capacity or default_capacity(params, self.n), device)
        self.ws = alloc_workspace(params, self.n, self.precision, device)
        # packed FP32 copies, one float4 per sorted particle (see dpd_bin_reorder)
        self.x32 = torch.empty((max(self.n, 1), 4), dtype=torch.float32, device=device)
        self.v32 = torch.empty((max(self.n, 1), 4), dtype=torch.float32, device=device)
        self.d_step = torch.zeros(1, dtype=torch.int64, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)
        self.stats = torch.zeros(2, dtype=torch.float64, device=device)

    # -- setup ----------------------------------------------------------
    def load(self, x, v, tag, typ, step: int = 0) -> None:
        """Copy host arrays in, reorder, build the list and compute F(step)."""
        src = State.empty(self.n, self.device)
        src.x.copy_(torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)))
        src.v.copy_(torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64)))
        src.tag.copy_(torch.as_tensor(np.ascontiguousarray(tag).astype(np.uint32).view(np.int32)))
        src.type.copy_(torch.as_tensor(np.ascontiguousarray(typ, dtype=np.uint8)))
        self.d_step.fill_(int(step))
        self.status.zero_()
        self.reorder_from(src)
        self.rebuild()
        self.fit_capacity()
        self.compute_forces(int(step))

    def fit_capacity(self, slack: float = 1.25) -> bool:
        """After a list build: if it overflowed, grow the list to the size the
        build reported (times slack) and build again.  Synchronises."""
        st = int(self.status.item())
        if not st & _abi.STATUS_NLIST_OVERFLOW:
            return False
        self.grow_nlist(slack)
        self.rebuild()
        st = int(self.status.item())
        if st & _abi.STATUS_NLIST_OVERFLOW:
            raise DPDError(_abi.DPD_ECAPACITY, "neighbour list still overflows after growing")
        return True

    def restore(self, x, v, f, tag, typ, step: int) -> None:
        """Resume from a snapshot of the sorted state (as ``host_state``
        returns it): no reordering and no force evaluation, so the next
        ``step`` continues the interrupted run bit for bit.  (The cell list,
        FP32 copies and neighbour list are rebuilt by that step; call
        ``reorder_from`` first to use ``rebuild`` / ``compute_forces`` on
        the restored state directly.)"""
        st = self.state
        st.x.copy_(torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)))
        st.v.copy_(torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64)))
        st.f.copy_(torch.as_tensor(np.ascontiguousarray(f, dtype=np.float64)))
        st.tag.copy_(torch.as_tensor(np.ascontiguousarray(tag).astype(np.uint32).view(np.int32)))
        st.type.copy_(torch.as_tensor(np.ascontiguousarray(typ, dtype=np.uint8)))
        self.d_step.fill_(int(step))
        self.status.zero_()

    def reorder_from(self, src: State) -> None:
        mixed = self.precision == MIXED
        dpd_bin_reorder(self.params, src, self.state, self.cells, self.ws,
                        self.x32, self.v32 if mixed else None)

    def rebuild(self) -> None:
        dpd_build_neighbors(self.params, self.state, self.cells, self.x32, self.nlist, self.status,
                            self.ws)

    def compute_forces(self, step: int, pe_out=None, precision=None) -> None:
        prec = self.precision if precision is None else precision
        dpd_forces(self.params, prec, self.state, self.cells, self.nlist, step, self.state.f, self.ws,
                   x32=self.x32 if prec == MIXED else None, v32=self.v32 if prec == MIXED else None,
                   pe_out=pe_out, stats=self.stats, status=self.status)

    # -- time stepping --------------------------------------------------
    def step(self, n_steps: int, reductions: Optional[torch.Tensor] = None, phase_events=None) -> None:
        mixed = self.precision == MIXED
        dpd_step(self.params, self.precision, self.state, n_steps, self.d_step, self.cells, self.nlist,
                 self.status, self.ws, reductions=reductions,
                 x32=self.x32, v32=self.v32 if mixed else None, phase_events=phase_events)

    def advance(self, n_steps: int, reductions: Optional[torch.Tensor] = None, slack: float = 1.25,
                max_grow: int = 4) -> int:
        """``step`` with recovery from a neighbour-list overflow inside the
        call: the state entering the call is kept on the device; when the
        status word reports an overflow after the call, the state is put
        back, the list grown to the last build's size times ``slack`` (or
        the capacity times ``slack`` when that is larger) and the call run
        again, so the result equals an uninterrupted run with a large
        enough list bit for bit.  The status word is cleared before each
        attempt.  Synchronises once per attempt.  Returns the number of
        times the list was grown."""
        st = self.state
        snap = (st.x.clone(), st.v.clone(), st.f.clone(), st.tag.clone(), st.type.clone(),
                self.d_step.clone())
        for grown in range(max_grow + 1):
            self.status.zero_()
            self.step(n_steps, reductions=reductions)
            flags = int(self.status.item())
            if not flags & _abi.STATUS_NLIST_OVERFLOW:
                return grown
            if grown == max_grow:
                break
            for dst, src in zip((st.x, st.v, st.f, st.tag, st.type, self.d_step), snap):
                dst.copy_(src)
            need = int(self.nlist.offset[self.n].item())
            cap = int(max(need, self.nlist.capacity) * slack) + 1
            self.nlist = NList.empty(self.n, cap, self.device)
        raise DPDError(_abi.DPD_ECAPACITY, f"neighbour list still overflows after growing {max_grow} times")

    def check_status(self) -> int:
        st = int(self.status.item())
        if st & _abi.STATUS_NLIST_OVERFLOW:
            raise DPDError(_abi.DPD_ECAPACITY, "neighbour list overflow (grow the capacity)")
        if st & _abi.STATUS_BAD_BOND:
            raise DPDError(_abi.DPD_EINVAL, "bond partner without a particle")
        if st & _abi.STATUS_NONFINITE:
            raise DPDError(_abi.DPD_EINVAL, "non-finite totals")
        return st

    def grow_nlist(self, factor: float = 1.5) -> None:
        need = int(self.nlist.offset[self.n].item())
        self.nlist = NList.empty(self.n, int(max(need, self.nlist.capacity) * factor), self.device)
        self.status.zero_()

    @property
    def step_count(self) -> int:
        return int(self.d_step.item())

    # -- host views (tests, checkpoints) ---------------------------------
    def host_state(self):
        st = self.state
        return (st.x.cpu().numpy(), st.v.cpu().numpy(), st.f.cpu().numpy(),
                st.tag.cpu().numpy().view(np.uint32), st.type.cpu().numpy())

    def host_nlist(self):
        off = self.nlist.offset.cpu().numpy().astype(np.int64)
        return off, self.nlist.index[: int(off[-1])].cpu().numpy()


# ------------------------------------------------------------------ Batch --

@dataclass
class Tiles:
    """Launch shapes of the batched phases (mirrors dpd_tiles); 0 = default."""

    force_grid: int = 0
    nlist_waves: int = 0
    nlist_kind: int = 0

    def c(self) -> _abi.dpd_tiles:
        t = _abi.dpd_tiles()
        t.force_grid, t.nlist_waves, t.nlist_kind = int(self.force_grid), int(self.nlist_waves), int(self.nlist_kind)
        return t


class Batch:
    """Device buffers of a batch of independent systems plus its driver.

    ``params`` lists one Params per system (same r_c, skin, dt, lambda, s and
    n_types; no bonds), ``sizes`` their particle counts.  Arrays are the
    systems' arrays concatenated in order; tags are local to each system.
    """

    def __init__(self, params, sizes, precision: int = MIXED, capacity: Optional[int] = None, device="cuda",
                 stream=None):
        if len(params) != len(sizes) or not params:
            raise ValueError("one Params per system, at least one system")
        self.params = list(params)
        self.sizes = np.asarray(sizes, dtype=np.int64)
        self.n_sys = len(self.params)
        self.offsets = np.zeros(self.n_sys + 1, dtype=np.int64)
        self.offsets[1:] = np.cumsum(self.sizes)
        self.n = int(self.offsets[-1])
        self.precision = int(precision)
        self.device = device
        L = lib()
        tb = int(L.dpd_batch_table_bytes(self.n_sys, self.n))
        if tb == 0:
            raise DPDError(_abi.DPD_EINVAL, "dpd_batch_table_bytes")
        self.table = torch.empty(tb, dtype=torch.uint8, device=device)
        arr = (_abi.dpd_params * self.n_sys)(*[p.c() for p in self.params])
        h = C.c_void_p()
        check(L.dpd_batch_create(arr, self.n_sys, self.offsets.ctypes.data, _ptr(self.table), tb,
                                 _stream(stream), C.byref(h)), "dpd_batch_create")
        self.handle = h
        n_tot, n_cells = C.c_int64(), C.c_int64()
        check(L.dpd_batch_sizes(self.handle, C.byref(n_tot), C.byref(n_cells)), "dpd_batch_sizes")
        self.n_cells = int(n_cells.value)
        nb = int(L.dpd_batch_workspace_bytes(self.handle, self.precision))
        if nb == 0:
            raise DPDError(_abi.DPD_EINVAL, "dpd_batch_workspace_bytes")
        self.ws = torch.empty(nb, dtype=torch.uint8, device=device)
        if capacity is None:
            capacity = sum(default_capacity(p, int(n)) for p, n in zip(self.params, self.sizes))
        self.state = State.empty(self.n, device)
        self.cells = Cells.empty(self.n, self.n_cells, device)
        self.nlist = NList.empty(self.n, capacity, device)
        self.x32 = torch.empty((self.n, 4), dtype=torch.float32, device=device)
        self.v32 = torch.empty((self.n, 4), dtype=torch.float32, device=device)
        self.d_step = torch.zeros(1, dtype=torch.int64, device=device)
        self.status = torch.zeros(1, dtype=torch.int32, device=device)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None and self.handle.value:
            torch.cuda.synchronize()
            lib().dpd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- tiles ----------------------------------------------------------
    def set_tiles(self, tiles: Tiles) -> None:
        t = tiles.c()
        check(lib().dpd_batch_set_tiles(self.handle, C.byref(t)), "dpd_batch_set_tiles")

    def get_tiles(self) -> Tiles:
        t = _abi.dpd_tiles()
        check(lib().dpd_batch_get_tiles(self.handle, C.byref(t)), "dpd_batch_get_tiles")
        return Tiles(int(t.force_grid), int(t.nlist_waves), int(t.nlist_kind))

    # -- setup ----------------------------------------------------------
    def load(self, x, v, tag, typ, step: int = 0) -> None:
        """Copy concatenated host arrays in, reorder, build the list and
        compute F(step)."""
        src = State.empty(self.n, self.device)
        src.x.copy_(torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64)))
        src.v.copy_(torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64)))
        src.tag.copy_(torch.as_tensor(np.ascontiguousarray(tag).astype(np.uint32).view(np.int32)))
        src.type.copy_(torch.as_tensor(np.ascontiguousarray(typ, dtype=np.uint8)))
        self.d_step.fill_(int(step))
        self.status.zero_()
        self.reorder_from(src)
        self.rebuild()
        self.fit_capacity()
        self.compute_forces(int(step))

    def reorder_from(self, src: State, stream=None) -> None:
        s_in, s_out, c = src.c(), self.state.c(), self.cells.c()
        mixed = self.precision == MIXED
        check(lib().dpd_batch_bin_reorder(self.handle, C.byref(s_in), C.byref(s_out), C.byref(c), _ptr(self.x32),
                                          _ptr(self.v32) if mixed else None, _ptr(self.ws), self.ws.numel(),
                                          _stream(stream)), "dpd_batch_bin_reorder")

    def rebuild(self, stream=None) -> None:
        s, c, n = self.state.c(), self.cells.c(), self.nlist.c()
        check(lib().dpd_batch_build_neighbors(self.handle, C.byref(s), C.byref(c), _ptr(self.x32), C.byref(n),
                                              _ptr(self.status), _ptr(self.ws), self.ws.numel(), _stream(stream)),
              "dpd_batch_build_neighbors")

    def fit_capacity(self, slack: float = 1.25) -> bool:
        st = int(self.status.item())
        if not st & _abi.STATUS_NLIST_OVERFLOW:
            return False
        need = int(self.nlist.offset[self.n].item())
        self.nlist = NList.empty(self.n, int(max(need, self.nlist.capacity) * slack), self.device)
        self.status.zero_()
        self.rebuild()
        if int(self.status.item()) & _abi.STATUS_NLIST_OVERFLOW:
            raise DPDError(_abi.DPD_ECAPACITY, "neighbour list still overflows after growing")
        return True

    def compute_forces(self, step: int, pe_out=None, precision=None, stream=None) -> None:
        prec = self.precision if precision is None else int(precision)
        s, c, n = self.state.c(), self.cells.c(), self.nlist.c()
        mixed = prec == MIXED
        check(lib().dpd_batch_forces(self.handle, prec, C.byref(s), C.byref(c), _ptr(self.x32) if mixed else None,
                                     _ptr(self.v32) if mixed else None, C.byref(n), int(step),
                                     _ptr(self.state.f), _ptr(pe_out), _ptr(self.status), _ptr(self.ws),
                                     self.ws.numel(), _stream(stream)), "dpd_batch_forces")

    # -- time stepping --------------------------------------------------
    def step(self, n_steps: int, reductions: Optional[torch.Tensor] = None, use_graph: bool = True,
             stream=None) -> None:
        """reductions: optional float64 [n_steps, n_sys, 8] device tensor."""
        if reductions is not None and tuple(reductions.shape) != (n_steps, self.n_sys, 8):
            raise ValueError("reductions must have shape (n_steps, n_sys, 8)")
        mixed = self.precision == MIXED
        s, c, n = self.state.c(), self.cells.c(), self.nlist.c()
        check(lib().dpd_batch_step(self.handle, self.precision, C.byref(s), int(n_steps), _ptr(self.d_step),
                                   _ptr(reductions), C.byref(c), C.byref(n), _ptr(self.x32),
                                   _ptr(self.v32) if mixed else None, _ptr(self.status), 1 if use_graph else 0,
                                   _ptr(self.ws), self.ws.numel(), _stream(stream)), "dpd_batch_step")

    def check_status(self) -> int:
        st = int(self.status.item())
        if st & _abi.STATUS_NLIST_OVERFLOW:
            raise DPDError(_abi.DPD_ECAPACITY, "neighbour list overflow (grow the capacity)")
        if st & _abi.STATUS_NONFINITE:
            raise DPDError(_abi.DPD_EINVAL, "non-finite totals")
        return st

    def system_slice(self, k: int) -> slice:
        return slice(int(self.offsets[k]), int(self.offsets[k + 1]))
