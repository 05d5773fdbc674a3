"""Throughput of the DPD hot path on one MI355X.

Workload: the amphiphile system of 16,000,000 particles at density 3 in a
cubic periodic box (side 174.716), 10% of the particles in H1T3 four-bead
chains (harmonic bonds k = 100, r0 = 0.7), a_ij = 25 like / 75 H-T and T-W /
35 H-W, gamma = 4.5, sigma = 3, dt = 0.01, s = 1/2, synthetic and seeded.

One timed step = velocity-Verlet phase 1, binning + reordering, ordered
neighbour list, pair + bond forces, phase 2 + statistics (every row of the
hot path).  Both precisions are run; the headline value is the mixed form's
particle-steps/s, the FP64 form sits beside it.  Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import subprocess
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "DPD pair-force evals/s & particle-steps/s at 16M, mixed vs FP64, 1 MI355X"
HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 32 lanes x 2.4 GHz full-rate 32-bit
# lane operations (non-packed) per second, in units of 1e12: a SIMD issues
# one wave64 instruction per two clocks (the FP32 vector peak, 157.3 TFLOP/s,
# is this rate with an FMA counted as two flops)
VALU_PEAK_TSLOTS = 256 * 4 * 32 * 2.4e9 / 1e12
# Algorithmic lane slots of one pair evaluation (full-rate operations count
# 1; 32-bit integer products and transcendentals, a quarter of the rate,
# count 4).  Philox4x32-10: 20 products (80) + 40 two-input xors; the
# uniforms 4; Box-Muller log, sqrt, cos (12) + 2 products; geometry (minimum
# image or cell offset, r^2, 1/r or sqrt and divide, unit vector) 20 / 23;
# weights 5 / 6; the force (e.v, phi, components) 12; the row sum: three
# compensated two-sums (18, mixed) or three adds (3, FP64).
ALU_SLOTS_PER_PAIR = {"mixed": 193, "fp64": 182}
# Phases of a step as dpd_step's events bracket them.  "integrate" is timed
# between events 0 and 1 of step k plus events 4 to 5.  Without a skin the
# force pass's row epilogue ends each step (second
# half-kick, and the next step's half-kick and drift), so "forces" holds it
# and "integrate" only the first step's phase 1 and the statistics' final
# sums; otherwise one pass over the state ends a step and starts the next
# (events 0 to 1) and the last step's second half-kick runs alone (events 4
# to 5).
PHASES = ["integrate", "reorder", "nlist", "forces"]


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_traffic_amphiphile16M.json")
FORCE_SOURCES = [os.path.join(ROOT, "paper_1311_0402_amd", "csrc", f)
                 for f in ("k_force.hip", "dpd_common.h", "dpd_launch.h")]


def force_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in FORCE_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision):
    """HBM bytes per force launch from the committed FETCH_SIZE / WRITE_SIZE
    runs (calibrated against a plain copy), or None when there are none or
    the force kernel's sources changed since they were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != force_source_hash():
        return None
    k = rec.get("kernels", {}).get(precision)
    return None if k is None else float(k["bytes_per_launch"])


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def force_bytes(n, nnz, n_bond_ends, precision):
    """Algorithmic HBM bytes of one force launch (j-gathers served on chip).

    FP64: per particle x, v (48) + tag 4 + type 1 + row offset 4 + F write 24,
    plus 4 per list entry; mixed: x32, v32 (24) + cell 4 + tag 4 + type 1 +
    offset 4 + F 24, plus 4 per list entry.  Bonds: the particle's partner
    entry (8) and, per bond end, the partner's index (4) and position (24).
    """
    per = 81 if precision == "fp64" else 61
    return n * per + 4 * nnz + 8 * n + 28 * n_bond_ends


def vv_bytes(n, steps):
    """Algorithmic HBM bytes per step of the half-kicks the force pass's row
    epilogue does (no skin): R v_h 24, x 24, tag, type 5; W
    drifted x, v 48, tag, type 5; the last step of a call only R v 24, W v
    24."""
    return n * (106.0 * (steps - 1) + 48.0) / steps


def phase_bytes(n, nnz, n_bond_ends, precision, n_cells, steps, fused=False):
    """Algorithmic HBM bytes of each phase of one step (each datum once).

    integrate: R x, v, F (72), tag, type (5); W drifted x, v (48), tag, type
    (5) every step, plus the last step's lone second half-kick (R v, F 48, W
    v 24) spread over the steps.  With the half-kicks in the force pass
    (fused: either form without a skin) the phase is the first step's
    phase 1 alone, and the forces phase adds vv_bytes.
    reorder: bin R x 24, W key, slot, cell 12; scan ~8 per cell; place R key,
    slot, tag 12, W tag, source 8; finalize R source, key 8, cell bounds 8,
    in-cell tags 12, x, v 48, type, cell 5, W x, v 48, tag, type, cell,
    perm, idx_of_tag 17, float4 copies 16 (+16 mixed).
    nlist: R x32 16, cell 4, cell table and ranks 8 per cell; W row count 4,
    4 per entry; scan 8.
    forces: see force_bytes.
    """
    mixed = precision == "mixed"
    reorder = n * (36 + 20 + 8 + 8 + 12 + 53 + 65 + 16 + (16 if mixed else 0)) + 8 * n_cells
    forces = float(force_bytes(n, nnz, n_bond_ends, precision))
    return {"integrate": 130.0 * n / steps if fused else 130.0 * n + 72.0 * n / steps,
            "reorder": float(reorder),
            "nlist": float(n * (16 + 4 + 4 + 8) + 4 * nnz + 8 * n_cells),
            "forces": forces + (vv_bytes(n, steps) if fused else 0.0)}


def alu_roofline(form, precision):
    """The force pass against the VALU issue peak: algorithmic lane slots of
    one evaluation per unique pair (Newton's third law) per second."""
    ach = form["unique_pairs_per_step"] * ALU_SLOTS_PER_PAIR[precision] / (form["force_ms"] * 1e-3) / 1e12
    return {"bound": "alu", "achieved": ach, "peak": VALU_PEAK_TSLOTS, "unit": "Tslot/s",
            "frac": ach / VALU_PEAK_TSLOTS, "slots_per_unique_pair": ALU_SLOTS_PER_PAIR[precision]}


def run_precision(P, torch, sysd, precision, steps, warmup, skin=0.0):
    """One form's timed step loop.  With skin > 0 the lists are built at
    r_c + skin and rebuilt only on steps where some particle has moved more
    than skin / 2 since the last rebuild; the reorder and list phases' bytes
    are then counted for the steps that rebuilt."""
    import paper_1311_0402_amd as PK
    prec = PK.FP64 if precision == "fp64" else PK.MIXED
    params = P.Params.like(sysd, skin=skin)
    sim = P.System(params, sysd.n, prec)
    sim.load(sysd.x, sysd.v, sysd.tag, sysd.type, step=0)
    torch.cuda.synchronize()
    sim.check_status()
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.check_status()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(6 * steps)]
    for e in evs:                       # materialise the HIP events
        e.record()
    red = torch.zeros((steps, 8), dtype=torch.float64, device="cuda")
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_start.record()
    sim.step(steps, reductions=red, phase_events=evs)
    t_stop.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    sim.check_status()
    total_ms = t_start.elapsed_time(t_stop)
    # windows between consecutive events of each step: phase 1 (with the
    # previous step's phase 2), reorder, list, forces, lone phase 2
    win = np.zeros(5)
    for k in range(steps):
        for ph in range(5):
            win[ph] += evs[6 * k + ph].elapsed_time(evs[6 * k + ph + 1])
    win /= steps
    phase_ms = np.array([win[0] + win[4], win[1], win[2], win[3]])
    r = red.cpu().numpy()
    nnz = int(sim.nlist.offset[sysd.n].item())
    n_bond_ends = 0 if sysd.partner is None else int((sysd.partner >= 0).sum())
    pairs = float(r[:, 5].mean())
    ms = total_ms / steps
    # without a skin the step's half-kicks run in the force pass's row
    # epilogue: its launch moves their bytes too
    fused = skin == 0
    n_cells = int(np.prod(P.cell_grid(params)))
    pb = phase_bytes(sysd.n, nnz, n_bond_ends, precision, n_cells, steps, fused)
    if skin > 0:
        # with a skin the force pass reads the filtered rows: the ordered
        # pairs inside r_c, not the list built at r_c + skin
        pb["forces"] = float(force_bytes(sysd.n, int(round(2 * pairs)), n_bond_ends, precision))
    fb = pb["forces"]
    rebuilt = float(r[:, 7].mean())
    pb["reorder"] *= rebuilt
    pb["nlist"] *= rebuilt
    if skin > 0:
        # every step's filter: R the list's entries 4 each, W the kept
        # entries 4 each, row counts and their scan ~12 per particle
        pb["nlist"] += 4.0 * nnz + 8.0 * pairs + 12.0 * sysd.n
    hbm_frac = {k: pb[k] / (phase_ms[q] * 1e-3) / 1e9 / HBM_PEAK_GBS for q, k in enumerate(PHASES)}
    # algorithmic bytes can only exceed what HBM moves if a phase's window
    # were mis-attributed (or its data served from cache)
    assert all(v <= 1.0 for v in hbm_frac.values()), hbm_frac
    out = {
        "ms_per_step": ms,
        "wall_s": wall,
        "particle_steps_per_s": sysd.n / (ms * 1e-3),
        "pair_evals_per_s": pairs / (phase_ms[3] * 1e-3),       # unique pairs / force time
        "ordered_pair_evals_per_s": 2 * pairs / (phase_ms[3] * 1e-3),
        "unique_pairs_per_step": pairs,
        "nnz": nnz,
        "phase_ms": {k: float(v) for k, v in zip(PHASES, phase_ms)},
        "force_ms": float(phase_ms[3]),
        "force_bytes": fb,
        # of which the step's half-kicks in the force pass's row epilogue
        "force_bytes_half_kicks": vv_bytes(sysd.n, steps) if fused else 0.0,
        "phase_gbs": {k: pb[k] / (phase_ms[q] * 1e-3) / 1e9 for q, k in enumerate(PHASES)},
        "phase_hbm_frac": hbm_frac,
        "kbt_last": float(r[-1, 6]),
        "momentum_max": float(np.abs(r[:, :3]).max()),
        "skin": skin,
        "rebuild_fraction": rebuilt,
    }
    out["force_alu_frac"] = alu_roofline(out, precision)["frac"]
    # the state the timed loop leaves (its forces are checked against the
    # oracle in the CPU leg): sorted x, v, F, tags, types and the step counter
    final = sim.host_state() + (sim.step_count,)
    del sim
    torch.cuda.empty_cache()
    return out, final


def run_batched(P, torch, steps, warmup, seq_steps, n_sys=256):
    """Replica ensemble: n_sys independent fluids of log-uniform size in
    [1000, 64000] at density 3, mixed precision.  The batch advances as one
    captured HIP graph per step (tiles from the autotuner); the comparison
    runs the same systems one after another, each with its own dpd_step."""
    import dpd_inputs as di
    from paper_1311_0402_amd import autotune
    spec = di.batched_spec(n_sys=n_sys, seed=4)
    systems = di.batched_systems(spec, seed=5)
    n_tot = int(sum(s.n for s in systems))
    b = P.Batch([P.Params.like(s) for s in systems], [s.n for s in systems], precision=P.MIXED)
    b.load(np.concatenate([s.x for s in systems], axis=1), np.concatenate([s.v for s in systems], axis=1),
           np.concatenate([s.tag for s in systems]), np.concatenate([s.type for s in systems]))
    torch.cuda.synchronize()
    b.check_status()
    t0 = time.perf_counter()
    tiles, timings = autotune.tune(b, use_cache=False)
    tune_s = time.perf_counter() - t0
    b.step(warmup, use_graph=True)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    b.step(steps, use_graph=True)
    e1.record()
    torch.cuda.synchronize()
    b.check_status()
    ms = e0.elapsed_time(e1) / steps
    b.close()
    del b
    torch.cuda.empty_cache()
    # the same systems one after another
    sims = []
    for s in systems:
        sim = P.System(P.Params.like(s), s.n, P.MIXED)
        sim.load(s.x, s.v, s.tag, s.type)
        sims.append(sim)
    for sim in sims:
        sim.step(2)
    torch.cuda.synchronize()
    e0.record()
    for sim in sims:
        sim.step(seq_steps)
    e1.record()
    torch.cuda.synchronize()
    for sim in sims:
        sim.check_status()
    ms_seq = e0.elapsed_time(e1) / seq_steps
    del sims
    torch.cuda.empty_cache()
    return {"n_sys": n_sys, "n_total": n_tot, "steps": steps, "ms_per_step": ms,
            "particle_steps_per_s": n_tot / (ms * 1e-3),
            "tiles": {"force_grid": tiles.force_grid, "nlist_waves": tiles.nlist_waves,
                      "nlist_kind": tiles.nlist_kind},
            "autotune_s": tune_s, "autotune_ms_per_step": timings,
            "sequential": {"steps": seq_steps, "ms_per_step": ms_seq,
                           "particle_steps_per_s": n_tot / (ms_seq * 1e-3)},
            "speedup_vs_sequential": ms_seq / ms}


def _time_ms(torch, fn, reps=5):
    """Median milliseconds of fn() over reps, HIP events on the current stream."""
    out = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        out.append(e0.elapsed_time(e1))
    return float(np.median(out))


def run_border(P, torch, sysd):
    """One GPU's share of the border exchange on the workload's own state:
    the send lists of the six faces of the box (band width r_c: the
    particles a neighbouring brick would need as ghosts), the 56-byte ghost
    records packed (position shifted by the face's periodic image), and the
    records unpacked into a ghost state.  Algorithmic bytes: lists 24 per
    particle (x) + 2 (flags) + 4 per listed entry; pack 113 per record
    (index, x, v, tag, type read; record written); unpack 109 per record."""
    n = sysd.n
    st = P.State.empty(n)
    st.x.copy_(torch.as_tensor(np.ascontiguousarray(sysd.x)))
    st.v.copy_(torch.as_tensor(np.ascontiguousarray(sysd.v)))
    st.tag.copy_(torch.as_tensor(np.ascontiguousarray(sysd.tag).astype(np.uint32).view(np.int32)))
    st.type.copy_(torch.as_tensor(np.ascontiguousarray(sysd.type, dtype=np.uint8)))
    lo, hi = np.zeros(3), np.asarray(sysd.box, dtype=np.float64)
    width = float(sysd.r_c)
    off = torch.zeros(7, dtype=torch.int32, device="cuda")
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = P.border_workspace(n)
    probe = torch.empty(1, dtype=torch.int32, device="cuda")
    P.dpd_border_lists(st, lo, hi, width, 63, off, probe[:0], status, ws)     # sizes only
    total = int(off[6].item())
    idx = torch.empty(total, dtype=torch.int32, device="cuda")
    status.zero_()
    rec = P.ghost_records(total)
    shift = np.zeros((6, 3))
    for d in range(3):
        shift[2 * d, d], shift[2 * d + 1, d] = hi[d], -hi[d]      # low face -> image above, high -> below
    ghosts = P.State.empty(total)
    count = off[6:7]
    t_lists = _time_ms(torch, lambda: P.dpd_border_lists(st, lo, hi, width, 63, off, idx, status, ws))
    t_pack = _time_ms(torch, lambda: P.dpd_border_pack(st, off, idx, shift, rec, status))
    t_unpack = _time_ms(torch, lambda: P.dpd_border_unpack(rec, count, ghosts, 0, status))
    torch.cuda.synchronize()
    assert int(status.item()) == 0, int(status.item())
    b_lists, b_pack, b_unpack = 26.0 * n + 4.0 * total, 113.0 * total, 109.0 * total
    out = {"n": n, "records": total, "faces": 6, "width": width,
           "ms": {"lists": t_lists, "pack": t_pack, "unpack": t_unpack},
           "gbs": {"lists": b_lists / (t_lists * 1e-3) / 1e9, "pack": b_pack / (t_pack * 1e-3) / 1e9,
                   "unpack": b_unpack / (t_unpack * 1e-3) / 1e9}}
    out["hbm_frac"] = {k: v / HBM_PEAK_GBS for k, v in out["gbs"].items()}
    del st, ghosts, rec, idx, ws
    torch.cuda.empty_cache()
    return out


def run_numerics(P, torch, n_tags=4_000_000, pairs=16, chain=4096):
    """The paper's numerics against the device library (A/B): one wave's
    dependent chain per function (shader clocks per call), and pair-Gaussian
    throughput of Philox4x32-10 + library log/sqrt/cos (the FP64 force
    pass's generator) against TEA-4 on signatures + the fast log and cosine."""
    from paper_1311_0402_amd import _abi
    from paper_1311_0402_amd import dpd as D
    names = {"log": _abi.FN_LOG, "fast_log": _abi.FN_FASTLOG, "cos2pi": _abi.FN_COS2PI,
             "fast_cos2pi": _abi.FN_FASTCOS2PI, "pow": _abi.FN_POW, "fast_pow": _abi.FN_FASTPOW}
    D.math_latency(_abi.FN_LOG, 64)                                 # warm-up (code load)
    lat = {k: D.math_latency(f, chain) / chain for k, f in names.items()}
    rng = np.random.default_rng(5)
    tag = torch.as_tensor(np.arange(n_tags, dtype=np.uint32).view(np.int32), device="cuda")
    v = torch.as_tensor(rng.standard_normal((3, n_tags)), device="cuda")
    sig = D.tea_signatures(tag, v, 1, 7)
    sink = torch.empty(n_tags, dtype=torch.float64, device="cuda")
    thr = {}
    for gen, name in ((0, "philox_library"), (1, "tea_fast")):
        ms = _time_ms(torch, lambda: D.gaussian_throughput(gen, n_tags, pairs, 1, 7, sig if gen else None, sink))
        thr[name] = n_tags * pairs / (ms * 1e-3)
    t_sig = _time_ms(torch, lambda: D.tea_signatures(tag, v, 1, 7))
    return {"cycles_per_call": lat, "chain": chain, "gaussians_per_s": thr,
            "tea_signatures_per_s": n_tags / (t_sig * 1e-3), "pairs_per_thread": pairs, "n_tags": n_tags}


def run_adjoint(P, torch, steps=50, ckpt=10):
    """Force-matching loss over a 50-step trajectory of the 512,000-particle
    A/B mixture (checkpoints every 10 steps): forward and backward times,
    their ratio and the peak device memory of the backward pass."""
    import dpd_inputs as di
    from paper_1311_0402_amd import adjoint as A
    s = di.binary_mixture(n=512_000, seed=6)
    spec = A.TrajectorySpec(params=P.Params.like(s), tag=s.tag, type=s.type, steps=steps, checkpoint=ckpt)
    a_ref = float(np.random.default_rng(7).uniform(25.0, 50.0))
    x0 = torch.tensor(s.x, device="cuda")
    v0 = torch.tensor(s.v, device="cuda")
    with torch.no_grad():
        T = A.trajectory_forces(torch.tensor([[25.0, a_ref], [a_ref, 25.0]], dtype=torch.float64),
                                torch.tensor(s.gamma), x0, v0, spec)
    out = {}
    for rep in range(2):                         # the first repetition warms up
        a = torch.tensor(s.a, dtype=torch.float64, requires_grad=True)
        g = torch.tensor(s.gamma, dtype=torch.float64, requires_grad=True)
        xr = x0.clone().requires_grad_(True)
        torch.cuda.synchronize()
        torch.cuda.reset_peak_memory_stats()
        t0 = time.perf_counter()
        loss = A.force_matching_loss(a, g, xr, v0, spec, T)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out = {"n": s.n, "steps": steps, "checkpoint": ckpt, "forward_s": t1 - t0, "backward_s": t2 - t1,
               "backward_over_forward": (t2 - t1) / (t1 - t0),
               "peak_device_bytes": int(torch.cuda.max_memory_allocated()),
               "loss": float(loss.item()), "grad_a_AB": float(a.grad[0, 1].item())}
    del T, x0, v0
    torch.cuda.empty_cache()
    return out


COPY_BYTES = 1 << 30


def run_counters(P, torch, sysd):
    """Two steps per precision (the kernels whose counters are read), then a
    plain device-to-device copy of COPY_BYTES whose FETCH_SIZE / WRITE_SIZE
    calibrate the counters against bytes actually moved."""
    for prec in (P.FP64, P.MIXED):
        sim = P.System(P.Params.like(sysd), sysd.n, prec)
        sim.load(sysd.x, sysd.v, sysd.tag, sysd.type, step=0)
        sim.step(2)
        torch.cuda.synchronize()
        sim.check_status()
        log(f"counters: precision {prec} nnz {int(sim.nlist.offset[sysd.n].item())}")
        del sim
        torch.cuda.empty_cache()
    src = torch.ones(COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"counters: copied {COPY_BYTES} bytes")
    print(json.dumps({"counters_run": True, "copy_bytes": COPY_BYTES}), flush=True)


# The paper's own speedup, quoted as context beside the oracle comparison.
PAPER_CONTEXT = {
    "speedup": "10-30x (best above 30x, at 2 million particles)",
    "gpu": "one NVIDIA K20X (Kepler, 1.31 TFLOP/s FP64, 250 GB/s)",
    "cpu": "all 16 cores of one AMD Opteron 6274 at 2.2 GHz (LAMMPS with the authors' DPD pair style)",
    "workload": "DPD fluids at density 3, 6 and 50, r_c 1 and 1.5, 8,192 to 2 million particles, "
                "neighbour list every 5 steps",
    "source": "abstract and Sec. 4.3",
}

# A child process with its own OpenMP thread count (the oracle fixes its
# thread count when it first runs): O(N^2) steps of the 3,000-particle fluid
# and the 64,000-particle channel, and, when the brute-force step is too long
# to run whole on one thread, the brute-force rows and forces of a bounded
# sample of rows (the per-step cost is the sample's times N / rows).
ORACLE_CHILD = r"""
import json, sys, time
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
import dpd_inputs as di
whole_64k = sys.argv[2] == "1"
out = {}
for name, s in (("fluid3000", di.small_fluid(1)), ("channel64000", di.poiseuille(seed=9))):
    f, _, _ = oracle.forces(s, s.x, s.v, s.tag, s.type, 0, mode="cells")
    if name == "fluid3000" or whole_64k:
        reps = 3 if name == "fluid3000" else 1
        t0 = time.perf_counter()
        for k in range(reps):
            oracle.step(s, s.x, s.v, f, s.tag, s.type, 1, use_cells=False)
        el = (time.perf_counter() - t0) / reps
        out[name] = {"n": s.n, "s_per_step": el, "steps": reps, "sampled_rows": None}
    else:
        q = np.sort(np.random.default_rng(5).choice(s.n, size=1000, replace=False)).astype(np.int32)
        vh = s.v + 0.5 * s.dt * f
        t0 = time.perf_counter()
        nbr = oracle.neighbors(s.x, s.box, s.r_c, query=q)
        oracle.forces(s, s.x, vh, s.tag, s.type, 1, nbr=nbr, query=q)
        el = (time.perf_counter() - t0) * s.n / q.size
        out[name] = {"n": s.n, "s_per_step": el, "steps": 0, "sampled_rows": int(q.size)}
sub = di.amphiphile(n=100_000, seed=31)
f, _, _ = oracle.forces(sub, sub.x, sub.v, sub.tag, sub.type, 0, mode="cells")
t0 = time.perf_counter()
oracle.run(sub, sub.x, sub.v, f, sub.tag, sub.type, 0, 5, use_cells=True)
out["cells_amphiphile100000"] = {"n": sub.n, "s_per_step": (time.perf_counter() - t0) / 5, "steps": 5}
print(json.dumps(out))
"""


def _oracle_child(threads, whole_64k):
    env = dict(os.environ, OMP_NUM_THREADS=str(threads))
    res = subprocess.run([sys.executable, "-c", ORACLE_CHILD, ROOT, "1" if whole_64k else "0"], env=env,
                         capture_output=True, text=True, check=True)
    return json.loads(res.stdout.strip().splitlines()[-1])


def host_info():
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        affinity = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        affinity = None
    return {"cpu_model": model, "nproc": os.cpu_count(), "affinity_cpus": affinity}


def form_errors(oracle, sysd, final, precision, n_sample=1000, seed=12):
    """Forces of the state a timed loop left, on a seeded sample of rows,
    against the FP64 oracle at the same state (x, v_h = v - dt/2 F, step):
    FP64 the largest |dF_i| / S_i (S_i = sum of the magnitudes of the row's
    terms) and the sample's L2; mixed the sample's L2 relative to |F| and
    |dF_i| / rms |F| at the 99.99th percentile and at the maximum."""
    x, v, f, tag, typ, step = final
    q = np.sort(np.random.default_rng(seed).choice(sysd.n, size=n_sample, replace=False)).astype(np.int32)
    vh = v - 0.5 * sysd.dt * f
    nbr = oracle.neighbors(x, sysd.box, sysd.r_c, query=q)
    f_ref, _, _, scale = oracle.forces(sysd, x, vh, tag, typ, step, nbr=nbr, query=q, with_scale=True)
    fq = f[:, q]
    d = np.linalg.norm(fq - f_ref, axis=0)
    l2 = float(np.linalg.norm(fq - f_ref) / np.linalg.norm(f_ref))
    rms = float(np.sqrt(np.mean(np.sum(f_ref ** 2, axis=0))))
    out = {"rows": int(n_sample), "step": int(step), "l2_rel": l2}
    if precision == "fp64":
        out["max_rel_to_row_scale"] = float(np.max(d / scale))
        out["bar"] = "|dF_i| <= 1e-12 S_i"
    else:
        out["p9999_rel_to_rms"] = float(np.percentile(d / rms, 99.99))
        out["max_rel_to_rms"] = float(np.max(d / rms))
        out["bar"] = "L2 and 99.99th percentile <= 1e-5"
    return out


def cpu_baseline(sysd, finals, gpu_value):
    """The CPU leg: the FP64 oracle on the host (plain, untuned, cell-list
    neighbour search for the large systems, FP64 throughout).

    * value: whole oracle time steps of the benchmark workload itself (the
      16M amphiphile system), 3 steps on all host threads;
    * O(N^2) per-step times of the 3,000-particle fluid and the
      64,000-particle channel on all threads and on one thread (the one-thread
      64,000 step from a 1,000-row sample, scaled by N / rows);
    * the errors of the GPU forms against the oracle on the states their
      timed loops left (forms.*.error)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    errors = {}
    for prec, final in finals.items():
        t0 = time.perf_counter()
        errors[prec] = form_errors(oracle, sysd, final, prec)
        errors[prec]["oracle_s"] = time.perf_counter() - t0
        log(f"cpu leg: {prec} error {errors[prec]}")
    finals.clear()
    t0 = time.perf_counter()
    f0, _, _ = oracle.forces(sysd, sysd.x, sysd.v, sysd.tag, sysd.type, 0, mode="cells")
    t_force = time.perf_counter() - t0
    k = 3
    t0 = time.perf_counter()
    oracle.run(sysd, sysd.x, sysd.v, f0, sysd.tag, sysd.type, 0, k, use_cells=True)
    el = time.perf_counter() - t0
    del f0
    rate = sysd.n * k / el
    log(f"cpu leg: {sysd.n}-particle oracle {el / k:.2f} s/step on {threads} threads")
    all_threads = _oracle_child(threads, True)
    one_thread = _oracle_child(1, False)
    log(f"cpu leg: O(N^2) all threads {all_threads}; one thread {one_thread}")

    def per_step(d):
        return {name: {"n": r["n"], "s_per_step": r["s_per_step"],
                       "particle_steps_per_s": r["n"] / r["s_per_step"],
                       "measured": "whole steps" if r.get("sampled_rows") is None else
                       f"{r['sampled_rows']} rows (brute-force rows and forces), scaled by N / rows"}
                for name, r in d.items()}

    return {"value": rate, "unit": "particle-steps/s", "cores": threads, "kind": "oracle",
            "sample": f"{k} whole oracle time steps of the {sysd.n}-particle amphiphile workload itself "
                      f"(cell-list neighbour search, FP64, all {threads} threads), {el:.1f} s "
                      f"(+ {t_force:.1f} s for the starting forces)",
            "host": host_info(),
            "gpu_over_oracle": gpu_value / rate,
            "paper_context": PAPER_CONTEXT,
            "o_n2_all_threads": per_step({k2: v for k2, v in all_threads.items() if k2 != "cells_amphiphile100000"}),
            "o_n2_one_thread": per_step({k2: v for k2, v in one_thread.items() if k2 != "cells_amphiphile100000"}),
            "cells_one_thread": per_step({"amphiphile100000": one_thread["cells_amphiphile100000"]}),
            "errors": errors}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--n", type=int, default=16_000_000)
    ap.add_argument("--precision", choices=["both", "fp64", "mixed"], default="both")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--counters", action="store_true",
                    help="short run for hardware counters: 2 steps per precision, then a plain "
                         "device copy of COPY_BYTES as the counter calibration; prints no bench line")
    ap.add_argument("--batched-steps", type=int, default=500,
                    help="timed steps of the 256-system batch (the batched configuration's length)")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the border-exchange and numerics A/B measurements")
    ap.add_argument("--pair-mode", type=int, default=None,
                    help="pair evaluation (0 every entry, 1 pairs once, 2 pairs once in FP64 only; "
                         "default: the library's)")
    ap.add_argument("--skin", type=float, default=0.3,
                    help="the mixed form is also timed with this Verlet skin (0: not run)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is described but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    import dpd_inputs as di
    import paper_1311_0402_amd as P
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.pair_mode is not None:
        P.set_pair_evaluation(args.pair_mode)
    t0 = time.perf_counter()
    sysd = di.amphiphile(n=args.n, seed=3)
    log(f"generated {sysd.n} particles, box {sysd.box[0]:.3f}, in {time.perf_counter() - t0:.1f}s")
    if args.counters:
        run_counters(P, torch, sysd)
        return

    results = {}
    finals = {}
    for prec in (["fp64", "mixed"] if args.precision == "both" else [args.precision]):
        results[prec], finals[prec] = run_precision(P, torch, sysd, prec, args.steps, args.warmup)
        log(f"{prec}: {results[prec]['ms_per_step']:.3f} ms/step, phases {results[prec]['phase_ms']}")

    if args.skin > 0 and args.precision != "fp64":
        res_skin, _ = run_precision(P, torch, sysd, "mixed", args.steps, args.warmup, skin=args.skin)
        results[f"mixed_skin{args.skin:g}"] = res_skin
        log(f"mixed, skin {args.skin:g}: {res_skin['ms_per_step']:.3f} ms/step, rebuilt on "
            f"{100 * res_skin['rebuild_fraction']:.0f}% of steps, phases {res_skin['phase_ms']}")

    if not args.no_batched:
        results["batched"] = run_batched(P, torch, args.batched_steps, 10, max(5, args.batched_steps // 10))
        bt = results["batched"]
        log(f"batched: {bt['ms_per_step']:.3f} ms/step for {bt['n_total']} particles in {bt['n_sys']} systems "
            f"(tiles {bt['tiles']}); sequential {bt['sequential']['ms_per_step']:.3f} ms/step")

    if not args.no_extras:
        results["border"] = run_border(P, torch, sysd)
        bd = results["border"]
        log(f"border exchange: {bd['records']} records, ms {bd['ms']}, GB/s {bd['gbs']}")
        results["numerics_ab"] = run_numerics(P, torch)
        log(f"numerics A/B: {results['numerics_ab']}")

    if not args.no_adjoint:
        results["adjoint"] = run_adjoint(P, torch)
        ad = results["adjoint"]
        log(f"adjoint: forward {ad['forward_s']:.3f} s, backward {ad['backward_s']:.3f} s "
            f"(ratio {ad['backward_over_forward']:.2f}), peak {ad['peak_device_bytes'] / 2**30:.2f} GiB")

    head = results.get("mixed") or results["fp64"]
    head_name = "mixed" if "mixed" in results else "fp64"
    phase_ms = head["phase_ms"]
    dom = max(phase_ms, key=phase_ms.get)
    fb = head["force_bytes"]
    achieved = fb / (head["force_ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": "forces", "achieved": achieved, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(head_name),
                "algorithmic_bytes": fb,
                # without a skin the force launch also does the half-kicks (a1, a10)
                "algorithmic_bytes_half_kicks": head["force_bytes_half_kicks"],
                "kernel_name": ("k_force_mixed" if head_name == "mixed" else "k_force_fp64") + "<..., kVV = true>",
                "dominant_phase": dom,
                # the bound the counters show: VALU issue, against the
                # algorithmic work of each unique pair evaluated once
                "alu": alu_roofline(head, head_name)}
    line = {
        "metric": METRIC,
        "value": head["particle_steps_per_s"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head_name == "mixed" else "f64",
        "data": "synthetic (seeded amphiphile system)",
        "config": {"workload": f"amphiphile-{sysd.n}", "n": sysd.n, "box": float(sysd.box[0]),
                   "rho": 3.0, "chains": "10% H1T3, k=100, r0=0.7", "dt": 0.01, "s": 0.5,
                   "neighbour_list": "rebuilt every step, skin 0", "precision": head_name},
        "pair_evals_per_s": head["pair_evals_per_s"],
        "forms": results,
        "roofline": roofline,
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(sysd, finals, line["value"])
        for prec, err in cb.pop("errors").items():
            results[prec]["error"] = err
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
