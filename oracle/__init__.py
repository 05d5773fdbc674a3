"""Python face of the FP64 CPU oracle (``dpd_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by the smoke check and by
the benchmark's CPU-baseline leg.  The product package never imports it and
it imports nothing from the product package.

Each wrapper takes and returns numpy arrays in the library layout
(``float64[3, N]`` structure of arrays, ``uint32`` tags, ``uint8`` types)
and calls the C function of the same name; see ``dpd_oracle.c`` for the
paper passage each one follows.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "dpd_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
MAX_TYPES = 8


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (no FMA contraction, OpenMP)."""
    cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fno-fast-math",
           "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-unknown-pragmas",
           SRC, "-o", LIB + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB + ".tmp", LIB)
    return LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _declare(_lib)
    return _lib


class OrcParams(C.Structure):
    _fields_ = [
        ("box", C.c_double * 3),
        ("r_c", C.c_double),
        ("r_list", C.c_double),
        ("s", C.c_double),
        ("dt", C.c_double),
        ("lam", C.c_double),
        ("n_types", C.c_int32),
        ("a", C.c_double * (MAX_TYPES * MAX_TYPES)),
        ("gamma", C.c_double * (MAX_TYPES * MAX_TYPES)),
        ("sigma", C.c_double * (MAX_TYPES * MAX_TYPES)),
        ("seed", C.c_uint64),
        ("body_g", C.c_double),
        ("body_split", C.c_double),
        ("bond_k", C.c_double),
        ("bond_r0", C.c_double),
        ("partner", C.c_void_p),
    ]


P = C.c_void_p


def _declare(L):
    L.orc_philox4x32_10.argtypes = [P, P, P]
    L.orc_philox_batch.argtypes = [C.c_int64, P, P, P]
    L.orc_xi.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64]
    L.orc_xi.restype = C.c_double
    L.orc_xi_batch.argtypes = [C.c_int64, P, P, C.c_uint64, C.c_uint64, P]
    L.orc_cell_grid.argtypes = [P, C.c_double, P]
    L.orc_cell_grid.restype = C.c_int
    L.orc_morton_rank_table.argtypes = [P, P]
    L.orc_reorder.argtypes = [C.c_int32, P, P, P, C.c_double, P, P]
    L.orc_reorder.restype = C.c_int
    L.orc_neighbors_brute.argtypes = [C.c_int32, P, P, C.c_double, C.c_int32, P, P, P, C.c_int64]
    L.orc_neighbors_brute.restype = C.c_int64
    L.orc_neighbors_cells.argtypes = [C.c_int32, P, P, C.c_double, P, P, C.c_int64]
    L.orc_neighbors_cells.restype = C.c_int64
    L.orc_forces.argtypes = [P, C.c_int32, P, P, P, P, C.c_int32, P, P, P, C.c_uint64, P, P, P, P]
    L.orc_forces.restype = C.c_int
    L.orc_step.argtypes = [P, C.c_int32, P, P, P, P, P, C.c_uint64, C.c_int, P]
    L.orc_step.restype = C.c_int
    L.orc_run.argtypes = [P, C.c_int32, P, P, P, P, P, C.c_uint64, C.c_int32, C.c_int,
                          P, C.c_int32, C.c_int32, C.c_int32, C.c_int32, P, P]
    L.orc_run.restype = C.c_int
    L.orc_forces_vjp.argtypes = [P, C.c_int32, P, P, P, P, P, P, C.c_uint64, P, P, P, P, P]
    L.orc_forces_vjp.restype = C.c_int
    L.orc_border_lists.argtypes = [C.c_int32, P, P, P, C.c_double, C.c_int32, P, P]
    L.orc_border_lists.restype = C.c_int64
    L.orc_border_pack.argtypes = [C.c_int32, P, P, P, P, P, P, P, P, P, P, P]
    L.orc_border_pack.restype = None
    L.orc_tea.argtypes = [C.c_int32, P, P]
    L.orc_tea_sig_inputs.argtypes = [C.c_uint32, C.c_double, C.c_double, C.c_double, P]
    L.orc_tea_signatures.argtypes = [C.c_int32, P, P, C.c_uint64, C.c_uint64, P]
    L.orc_tea_xi_batch.argtypes = [C.c_int64, P, P, C.c_uint64, C.c_uint64, P, P]


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def params(sys_, *, skin: float = 0.0) -> OrcParams:
    """Oracle parameter block from a ``dpd_inputs.System``."""
    p = OrcParams()
    for k in range(3):
        p.box[k] = float(sys_.box[k])
    p.r_c = float(sys_.r_c)
    p.r_list = float(sys_.r_c + skin)
    p.s = float(sys_.s)
    p.dt = float(sys_.dt)
    p.lam = float(sys_.lam)
    nt = int(sys_.n_types)
    if nt < 1 or nt > MAX_TYPES:
        raise ValueError("n_types out of range")
    p.n_types = nt
    for name in ("a", "gamma", "sigma"):
        tab = np.asarray(getattr(sys_, name), dtype=np.float64).reshape(nt, nt)
        arr = getattr(p, name)
        for t in range(nt * nt):
            arr[t] = float(tab.reshape(-1)[t])
    p.seed = int(sys_.seed) & ((1 << 64) - 1)
    p.body_g = float(sys_.body_g)
    p.body_split = float(sys_.body_split)
    p.bond_k = float(sys_.bond_k)
    p.bond_r0 = float(sys_.bond_r0)
    p._partner_keep = None
    if sys_.partner is not None:
        part = _c(sys_.partner, np.int32).reshape(-1)
        p._partner_keep = part
        p.partner = part.ctypes.data
    else:
        p.partner = None
    return p


# ---------------------------------------------------------------- RNG ----

def philox(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    ctr = _c(ctr, np.uint32).reshape(-1, 4)
    key = _c(key, np.uint32).reshape(-1, 2)
    out = np.empty_like(ctr)
    lib().orc_philox_batch(ctr.shape[0], _ptr(ctr), _ptr(key), _ptr(out))
    return out


def xi(ti, tj, step: int, seed: int) -> np.ndarray:
    ti = _c(np.atleast_1d(ti), np.uint32)
    tj = _c(np.atleast_1d(tj), np.uint32)
    out = np.empty(ti.shape[0], dtype=np.float64)
    lib().orc_xi_batch(ti.shape[0], _ptr(ti), _ptr(tj), int(step), int(seed) & ((1 << 64) - 1), _ptr(out))
    return out


# ------------------------------------------------------ cells, reorder ----

def cell_grid(box, r_list: float):
    box = _c(box, np.float64)
    nc = np.zeros(3, dtype=np.int32)
    rc = lib().orc_cell_grid(_ptr(box), float(r_list), _ptr(nc))
    if rc != 0:
        raise ValueError("box too small for the cell grid (need >= 3 cells per side)")
    return nc


def morton_rank_table(nc) -> np.ndarray:
    nc = _c(nc, np.int32)
    rank = np.empty(int(np.prod(nc.astype(np.int64))), dtype=np.int32)
    lib().orc_morton_rank_table(_ptr(nc), _ptr(rank))
    return rank


def reorder(x, tag, box, r_list: float):
    """(perm new->old, cell_start) ordered by (Morton rank of cell, tag)."""
    x = _c(x, np.float64)
    tag = _c(tag, np.uint32)
    box = _c(box, np.float64)
    n = x.shape[1]
    nc = cell_grid(box, r_list)
    perm = np.empty(n, dtype=np.int32)
    cs = np.empty(int(np.prod(nc.astype(np.int64))) + 1, dtype=np.int32)
    rc = lib().orc_reorder(n, _ptr(x), _ptr(tag), _ptr(box), float(r_list), _ptr(perm), _ptr(cs))
    if rc != 0:
        raise ValueError("orc_reorder failed")
    return perm, cs


# ---------------------------------------------------------- neighbours ----

def neighbors(x, box, r_list: float, *, mode: str = "brute", query=None):
    """CSR (off int64[nq+1], idx int32[nnz]) of ascending neighbour rows."""
    x = _c(x, np.float64)
    box = _c(box, np.float64)
    n = x.shape[1]
    L = lib()
    if mode == "brute":
        q = None if query is None else _c(query, np.int32)
        nq = n if q is None else q.shape[0]
        count = np.empty(nq, dtype=np.int32)
        total = L.orc_neighbors_brute(n, _ptr(x), _ptr(box), float(r_list), nq, _ptr(q), _ptr(count), None, 0)
        idx = np.empty(max(total, 1), dtype=np.int32)
        L.orc_neighbors_brute(n, _ptr(x), _ptr(box), float(r_list), nq, _ptr(q), _ptr(count), _ptr(idx), total)
    elif mode == "cells":
        if query is not None:
            raise ValueError("cells mode builds all rows")
        count = np.empty(n, dtype=np.int32)
        total = L.orc_neighbors_cells(n, _ptr(x), _ptr(box), float(r_list), _ptr(count), None, 0)
        if total < 0:
            raise ValueError("cell grid invalid")
        idx = np.empty(max(total, 1), dtype=np.int32)
        L.orc_neighbors_cells(n, _ptr(x), _ptr(box), float(r_list), _ptr(count), _ptr(idx), total)
    else:
        raise ValueError(mode)
    off = np.zeros(count.shape[0] + 1, dtype=np.int64)
    np.cumsum(count, out=off[1:])
    return off, idx[:total]


# -------------------------------------------------------------- forces ----

def forces(sys_, x, v, tag, typ, step: int, *, nbr=None, query=None, skin: float = 0.0,
           mode: str = "brute", with_scale: bool = False):
    """Forces (float64[3, nq]), per-row PE halves and per-row pair counts
    (plus, with_scale, the per-row sum of term magnitudes)."""
    p = params(sys_, skin=skin)
    x = _c(x, np.float64)
    v = _c(v, np.float64)
    tag = _c(tag, np.uint32)
    typ = _c(typ, np.uint8)
    n = x.shape[1]
    if nbr is None:
        nbr = neighbors(x, sys_.box, p.r_list, mode=mode if query is None else "brute", query=query)
    off, idx = nbr
    off = _c(off, np.int64)
    idx = _c(idx, np.int32)
    q = None if query is None else _c(query, np.int32)
    nq = n if q is None else q.shape[0]
    f = np.empty((3, nq), dtype=np.float64)
    pe = np.empty(nq, dtype=np.float64)
    npair = np.empty(nq, dtype=np.int32)
    scale = np.empty(nq, dtype=np.float64) if with_scale else None
    lib().orc_forces(C.byref(p), n, _ptr(x), _ptr(v), _ptr(tag), _ptr(typ), nq, _ptr(q),
                     _ptr(off), _ptr(idx), int(step), _ptr(f), _ptr(pe), _ptr(npair), _ptr(scale))
    if with_scale:
        return f, pe, npair, scale
    return f, pe, npair


def step(sys_, x, v, f, tag, typ, step_next: int, *, use_cells: bool = False, skin: float = 0.0):
    """One velocity-Verlet step in place on copies; returns (x, v, f, red[8])."""
    p = params(sys_, skin=skin)
    x = np.array(x, dtype=np.float64, order="C", copy=True)
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    tag = _c(tag, np.uint32)
    typ = _c(typ, np.uint8)
    red = np.zeros(8, dtype=np.float64)
    rc = lib().orc_step(C.byref(p), x.shape[1], _ptr(x), _ptr(v), _ptr(f), _ptr(tag), _ptr(typ),
                        int(step_next), 1 if use_cells else 0, _ptr(red))
    if rc != 0:
        raise RuntimeError("orc_step failed")
    return x, v, f, red


def forces_vjp(sys_, x, v, tag, typ, step: int, g, *, nbr=None, skin: float = 0.0, mode="brute"):
    """(xbar, vbar, abar[nt,nt], gammabar[nt,nt]) for dL/dF = g."""
    p = params(sys_, skin=skin)
    x = _c(x, np.float64)
    v = _c(v, np.float64)
    g = _c(g, np.float64)
    tag = _c(tag, np.uint32)
    typ = _c(typ, np.uint8)
    n = x.shape[1]
    if nbr is None:
        nbr = neighbors(x, sys_.box, p.r_list, mode=mode)
    off, idx = _c(nbr[0], np.int64), _c(nbr[1], np.int32)
    nt = int(sys_.n_types)
    xb = np.empty((3, n)); vb = np.empty((3, n))
    ab = np.empty(nt * nt); gb = np.empty(nt * nt)
    lib().orc_forces_vjp(C.byref(p), n, _ptr(x), _ptr(v), _ptr(tag), _ptr(typ), _ptr(off),
                         _ptr(idx), int(step), _ptr(g), _ptr(xb), _ptr(vb), _ptr(ab), _ptr(gb))
    return xb, vb, ab.reshape(nt, nt), gb.reshape(nt, nt)


def run(sys_, x, v, f, tag, typ, step0: int, n_steps: int, *, use_cells: bool = True,
        profile=None, skin: float = 0.0):
    """n_steps oracle steps; returns (x, v, f, red[n_steps, 8], prof_mean or None).

    profile = (axis, component, nbins, from_step) averages that velocity
    component in slabs along the axis over the steps >= from_step.
    """
    p = params(sys_, skin=skin)
    x = np.array(x, dtype=np.float64, order="C", copy=True)
    v = np.array(v, dtype=np.float64, order="C", copy=True)
    f = np.array(f, dtype=np.float64, order="C", copy=True)
    tag = _c(tag, np.uint32)
    typ = _c(typ, np.uint8)
    red = np.zeros((n_steps, 8), dtype=np.float64)
    prof = cnt = None
    pa = pc = nb = pf = 0
    if profile is not None:
        pa, pc, nb, pf = profile
        prof = np.zeros(nb); cnt = np.zeros(nb)
    rc = lib().orc_run(C.byref(p), x.shape[1], _ptr(x), _ptr(v), _ptr(f), _ptr(tag), _ptr(typ),
                       int(step0), int(n_steps), 1 if use_cells else 0, _ptr(red),
                       pa, pc, nb, pf, _ptr(prof), _ptr(cnt))
    if rc != 0:
        raise RuntimeError("orc_run failed")
    prof_mean = None if prof is None else prof / np.maximum(cnt, 1.0)
    return x, v, f, red, prof_mean


# ------------------------------------------- TEA generator (A/B study) ----

def tea(rounds: int, v, key):
    """TEA cycles on the block (v0, v1) with key k[4]."""
    w = _c(v, np.uint32).copy()
    lib().orc_tea(int(rounds), _ptr(w), _ptr(_c(key, np.uint32)))
    return w


def tea_sig_inputs(tag: int, vx: float, vy: float, vz: float):
    out = np.zeros(2, dtype=np.uint32)
    lib().orc_tea_sig_inputs(int(tag) & 0xFFFFFFFF, float(vx), float(vy), float(vz), _ptr(out))
    return out


def tea_signatures(tag, v, step: int, seed: int):
    tag = _c(tag, np.uint32)
    v = _c(v, np.float64)
    sig = np.empty(tag.shape[0], dtype=np.uint32)
    lib().orc_tea_signatures(tag.shape[0], _ptr(tag), _ptr(v), int(step), int(seed) & ((1 << 64) - 1), _ptr(sig))
    return sig


def tea_xi(si, sj, step: int, seed: int):
    """(words uint32[n, 2], xi float64[n]) of TEA-4 on signature pairs."""
    si = _c(np.atleast_1d(si), np.uint32)
    sj = _c(np.atleast_1d(sj), np.uint32)
    n = si.shape[0]
    w = np.empty((n, 2), dtype=np.uint32)
    xi = np.empty(n, dtype=np.float64)
    lib().orc_tea_xi_batch(n, _ptr(si), _ptr(sj), int(step), int(seed) & ((1 << 64) - 1), _ptr(w), _ptr(xi))
    return w, xi


# ------------------------------------------------- border exchange ----

def border_lists(x, lo, hi, width: float, face_mask: int = 63):
    """(off int64[7], idx int32[total]): the ascending send list of every
    selected face of the brick [lo, hi) (Sec. 3.6, Algorithm 6)."""
    x = _c(x, np.float64)
    lo = _c(lo, np.float64)
    hi = _c(hi, np.float64)
    n = x.shape[1]
    off = np.zeros(7, dtype=np.int64)
    total = lib().orc_border_lists(n, _ptr(x), _ptr(lo), _ptr(hi), float(width), int(face_mask), _ptr(off), None)
    idx = np.empty(max(total, 1), dtype=np.int32)
    lib().orc_border_lists(n, _ptr(x), _ptr(lo), _ptr(hi), float(width), int(face_mask), _ptr(off), _ptr(idx))
    return off, idx[:total]


def border_pack(x, v, tag, typ, off, idx, shift):
    """Ghost records of the send lists: (gx float64[3, total], gv, gtag
    uint32[total], gtype uint32[total]); shift is float64[6, 3]."""
    x = _c(x, np.float64)
    v = _c(v, np.float64)
    tag = _c(tag, np.uint32)
    typ = _c(typ, np.uint8)
    off = _c(off, np.int64)
    idx = _c(idx, np.int32)
    shift = _c(shift, np.float64).reshape(6, 3)
    total = int(off[6])
    gx = np.empty((3, total)); gv = np.empty((3, total))
    gtag = np.empty(total, dtype=np.uint32); gtype = np.empty(total, dtype=np.uint32)
    if total:
        lib().orc_border_pack(x.shape[1], _ptr(x), _ptr(v), _ptr(tag), _ptr(typ), _ptr(off), _ptr(idx),
                              _ptr(shift), _ptr(gx), _ptr(gv), _ptr(gtag), _ptr(gtype))
    return gx, gv, gtag, gtype


def periodic_shifts(box):
    """Face shifts of a brick that spans the periodic box: a particle sent
    through the low face of axis d reappears at x_d + L_d, through the high
    face at x_d - L_d."""
    sh = np.zeros((6, 3))
    for d in range(3):
        sh[2 * d, d] = float(box[d])
        sh[2 * d + 1, d] = -float(box[d])
    return sh


def staged_halo(x, v, tag, typ, box, width: float):
    """The three-stage exchange on one periodic brick [0, L): the x faces
    over the owned particles, then the y faces over owned + x ghosts, then
    the z faces over all of them.  Returns (x, v, tag, type) of the owned
    particles followed by the ghosts, and the per-stage (off, idx)."""
    lo = np.zeros(3)
    hi = np.asarray(box, dtype=np.float64)
    sh = periodic_shifts(box)
    X, V = np.array(x, dtype=np.float64), np.array(v, dtype=np.float64)
    T, Y = np.array(tag, dtype=np.uint32), np.array(typ, dtype=np.uint8)
    stages = []
    for d in range(3):
        off, idx = border_lists(X, lo, hi, width, 3 << (2 * d))
        gx, gv, gt, gy = border_pack(X, V, T, Y, off, idx, sh)
        stages.append((off, idx))
        X = np.concatenate([X, gx], axis=1)
        V = np.concatenate([V, gv], axis=1)
        T = np.concatenate([T, gt])
        Y = np.concatenate([Y, gy.astype(np.uint8)])
    return X, V, T, Y, stages


# ------------------------------------------------- trajectory adjoint ----

def trajectory(sys_, x0, v0, steps: int, *, a=None, gamma=None, use_cells: bool = True):
    """States (x_k, v_k, F_k) for k = 0..steps, in the caller's (tag) order.

    F_0 = F(x0, v0, 0); each later state is one velocity-Verlet step
    (Eq (1), Algorithm 1's integration phases) with forces at step k.
    """
    s = _with_tables(sys_, a, gamma)
    tag, typ = sys_.tag, sys_.type
    f0, _, _ = forces(s, x0, v0, tag, typ, 0, mode="cells" if use_cells else "brute")
    out = [(np.array(x0, dtype=np.float64), np.array(v0, dtype=np.float64), f0)]
    x, v, f = out[0]
    for k in range(1, steps + 1):
        x, v, f, _ = step(s, x, v, f, tag, typ, k, use_cells=use_cells)
        out.append((x, v, f))
    return out


def _with_tables(sys_, a, gamma):
    import copy
    s = copy.copy(sys_)
    if a is not None:
        s.a = np.asarray(a, dtype=np.float64)
    if gamma is not None:
        s.gamma = np.asarray(gamma, dtype=np.float64)
    return s


def force_matching_grad(sys_, x0, v0, steps: int, targets, *, a=None, gamma=None, use_cells: bool = True):
    """Loss L = sum_{k=1..steps} |F_k - T_k|^2 and its gradient with respect
    to (a, gamma, x0, v0), pair Gaussian and pair sets held fixed.

    Reverse of each step (c = dt/2, lambda = 1/2, v~ = v_h):
      Fb_k += 2 (F_k - T_k);  Fb_k += c vb_k;
      (xPhi, vPhi, aPhi, gPhi) = VJP of F at (x_k, v_h,k, step k) with Fb_k;
      xt = xb_k + xPhi;  vh = vb_k + vPhi + dt xt;
      xb_{k-1} = xt;  vb_{k-1} = vh;  Fb_{k-1} = c vh.
    Finally the VJP of F_0 = F(x0, v0, 0) with Fb_0.  Returns
    (L, abar, gammabar, xbar0, vbar0).
    """
    s = _with_tables(sys_, a, gamma)
    tag, typ = sys_.tag, sys_.type
    traj = trajectory(sys_, x0, v0, steps, a=a, gamma=gamma, use_cells=use_cells)
    T = np.asarray(targets, dtype=np.float64)
    loss = sum(float(np.sum((traj[k][2] - T[k - 1]) ** 2)) for k in range(1, steps + 1))
    c = 0.5 * s.dt
    nt = int(s.n_types)
    gx = np.zeros_like(traj[0][0]); gv = np.zeros_like(gx); gf = np.zeros_like(gx)
    ga = np.zeros((nt, nt)); gg = np.zeros((nt, nt))
    mode = "cells" if use_cells else "brute"
    for k in range(steps, 0, -1):
        xk, vk, fk = traj[k]
        _, vprev, fprev = traj[k - 1]
        gf = gf + 2.0 * (fk - T[k - 1])
        gf_eff = gf + c * gv
        vh = vprev + c * fprev                      # the velocity F_k was evaluated with
        xb, vb, ab, gb = forces_vjp(s, xk, vh, tag, typ, k, gf_eff, mode=mode)
        xt = gx + xb
        vh_bar = gv + vb + s.dt * xt
        gx, gv, gf = xt, vh_bar, c * vh_bar
        ga += ab; gg += gb
    xb, vb, ab, gb = forces_vjp(s, traj[0][0], traj[0][1], tag, typ, 0, gf, mode=mode)
    return loss, ga + ab, gg + gb, gx + xb, gv + vb
