"""Pins of the CPU oracle against things other than itself.

Each test ties one oracle function to a fact fixed by the paper or by
mathematics: an independent library implementation, a closed form, an
invariant, a special case, or brute force.  A plausible slip in the oracle
(dropped term, wrong sign, transposed index) fails at least one of these.
"""
import json
import os
import subprocess
import tempfile

import numpy as np
import pytest

import dpd_inputs as di
import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- Philox --

_PHILOX_PROBE = r"""
#include <ATen/core/PhiloxRNGEngine.h>
#include <cstdio>
#include <cstdint>
int main() {
  unsigned long long c0, c1, c2, c3, k0, k1;
  while (std::scanf("%llu %llu %llu %llu %llu %llu", &c0, &c1, &c2, &c3, &k0, &k1) == 6) {
    // torch's engine: key = seed words, counter = (offset lo, offset hi,
    // subsequence lo, subsequence hi)
    at::Philox4_32 eng((uint64_t)k0 | ((uint64_t)k1 << 32),
                       (uint64_t)c2 | ((uint64_t)c3 << 32),
                       (uint64_t)c0 | ((uint64_t)c1 << 32));
    uint32_t w0 = eng(), w1 = eng(), w2 = eng(), w3 = eng();
    std::printf("%u %u %u %u\n", w0, w1, w2, w3);
  }
}
"""


def _torch_include():
    import torch
    return os.path.join(os.path.dirname(torch.__file__), "include")


def test_philox_matches_independent_engine():
    """Oracle Philox4x32-10 == torch's header-only Philox engine (called, not copied)."""
    rng = np.random.default_rng(123)
    ctr = rng.integers(0, 2**32, size=(512, 4), dtype=np.uint64).astype(np.uint32)
    key = rng.integers(0, 2**32, size=(512, 2), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0; key[0] = 0
    ctr[1] = 0xFFFFFFFF; key[1] = 0xFFFFFFFF
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "p.cpp")
        exe = os.path.join(td, "p")
        with open(src, "w") as fh:
            fh.write(_PHILOX_PROBE)
        subprocess.run(["g++", "-O1", "-std=c++17", "-I", _torch_include(), src, "-o", exe], check=True)
        inp = "\n".join(" ".join(str(int(v)) for v in list(c) + list(k)) for c, k in zip(ctr, key))
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    ref = np.array([[int(t) for t in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)
    got = oracle.philox(ctr, key).astype(np.uint64)
    np.testing.assert_array_equal(got, ref)


# -------------------------------------------------------------------- xi --

def test_xi_symmetric_and_step_dependent():
    rng = np.random.default_rng(5)
    ti = rng.integers(0, 10**6, 1000).astype(np.uint32)
    tj = rng.integers(0, 10**6, 1000).astype(np.uint32)
    a = oracle.xi(ti, tj, 17, 99)
    b = oracle.xi(tj, ti, 17, 99)
    np.testing.assert_array_equal(a, b)                    # xi_ij = xi_ji (Sec. 3.5)
    c = oracle.xi(ti, tj, 18, 99)
    d = oracle.xi(ti, tj, 17, 100)
    assert np.mean(a == c) < 0.01 and np.mean(a == d) < 0.01


def test_xi_box_muller_from_words():
    """xi equals the z_1 Box-Muller form of the Philox words (Sec. 3.5),
    computed here from the engine words with numpy's own log/cos."""
    ti = np.array([3, 10, 7, 123456], dtype=np.uint32)
    tj = np.array([9, 2, 7 + 1, 42], dtype=np.uint32)
    step, seed = (1 << 33) + 5, 0x1234_5678_9ABC_DEF0
    lo, hi = np.minimum(ti, tj), np.maximum(ti, tj)
    ctr = np.stack([lo, hi, np.full(4, step & 0xFFFFFFFF), np.full(4, step >> 32)], axis=1)
    key = np.tile(np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint64), (4, 1))
    w = oracle.philox(ctr.astype(np.uint32), key.astype(np.uint32)).astype(np.float64)
    u1 = (w[:, 0] + 0.5) / 2.0**32
    u2 = w[:, 1] / 2.0**32
    expect = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    np.testing.assert_allclose(oracle.xi(ti, tj, step, seed), expect, rtol=1e-14, atol=1e-14)


def test_xi_moments_standard_normal():
    """Moments 1..4 of xi over 2^20 pairs: 0, 1, 0, 3 within sampling error
    (the paper's moment check of its generator, Sec. 3.5)."""
    n = 1 << 20
    rng = np.random.default_rng(9)
    ti = rng.integers(0, 65536, n).astype(np.uint32)
    tj = (ti + 1 + rng.integers(0, 65535, n)).astype(np.uint32)
    z = oracle.xi(ti, tj, 1000, 2024)
    se = 1.0 / np.sqrt(n)
    assert abs(z.mean()) < 5 * se
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0) * se
    assert abs(np.mean(z**3)) < 5 * np.sqrt(15.0) * se
    assert abs(np.mean(z**4) - 3.0) < 5 * np.sqrt(96.0) * se
    # no lag correlation over consecutive steps or consecutive partners
    z2 = oracle.xi(ti, tj, 1001, 2024)
    z3 = oracle.xi(ti, tj + 1, 1000, 2024)
    assert abs(np.corrcoef(z, z2)[0, 1]) < 5 * se
    assert abs(np.corrcoef(z, z3)[0, 1]) < 5 * se


# ------------------------------------------------------- pair force pins --

def _pair_system(xi_, xj, vi, vj, *, a=25.0, gamma=4.5, sigma=3.0, s=0.5, dt=0.01,
                 box=(6.0, 6.0, 6.0), ti=0, tj=1, seed=11):
    x = np.array([xi_, xj], dtype=np.float64).T.copy()
    v = np.array([vi, vj], dtype=np.float64).T.copy()
    sy = di.System(box=np.array(box, dtype=np.float64), x=x, v=v,
                   tag=np.array([ti, tj], dtype=np.uint32), type=np.zeros(2, dtype=np.uint8),
                   a=np.array([[a]]), gamma=np.array([[gamma]]), sigma=np.array([[sigma]]),
                   s=s, dt=dt, seed=seed)
    return sy


def test_two_particle_closed_form_golden():
    g = json.load(open(os.path.join(GOLDEN, "two_particle.json")))
    pr = g["params"]
    sy = _pair_system([2.5, 3.0, 3.0], [2.0, 3.0, 3.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0],
                      a=pr["a"], gamma=pr["gamma"], sigma=0.0, s=pr["s"], dt=pr["dt"])
    f, pe, npair = oracle.forces(sy, sy.x, sy.v, sy.tag, sy.type, 7)
    np.testing.assert_allclose(f[:, 0], [g["F_C"] + g["F_D"], 0, 0], rtol=1e-15, atol=1e-15)
    np.testing.assert_allclose(f[:, 1], [-(g["F_C"] + g["F_D"]), 0, 0], rtol=1e-15, atol=1e-15)
    assert list(npair) == [1, 1]
    # potential 1/2 a r_c w_C^2, split half / half
    np.testing.assert_allclose(pe, [0.25 * 25 * 0.25] * 2, rtol=1e-15)
    # random part alone: sigma w_R xi / sqrt(dt) along e, xi from the pinned generator
    sy2 = _pair_system([2.5, 3.0, 3.0], [2.0, 3.0, 3.0], [1.0, 0.0, 0.0], [0.0, 0.0, 0.0],
                       a=0.0, gamma=0.0, sigma=pr["sigma"], s=pr["s"], dt=pr["dt"])
    f2, _, _ = oracle.forces(sy2, sy2.x, sy2.v, sy2.tag, sy2.type, 7)
    xi_ = oracle.xi([0], [1], 7, sy2.seed)[0]
    np.testing.assert_allclose(f2[0, 0], g["F_R_over_xi"] * xi_, rtol=1e-14)
    np.testing.assert_allclose(f2[1:, 0], 0.0, atol=1e-15)
    for case in g["cases"]:
        sy3 = _pair_system([2.0 + case["r"], 3.0, 3.0], [2.0, 3.0, 3.0],
                           [case["e_dot_v"], 0.0, 0.0], [0.0, 0.0, 0.0],
                           a=case["a"], gamma=case["gamma"], sigma=0.0, s=case["s"])
        f3, _, _ = oracle.forces(sy3, sy3.x, sy3.v, sy3.tag, sy3.type, 1)
        np.testing.assert_allclose(f3[0, 0], case["F_C"] + case["F_D"], rtol=1e-14, atol=1e-14)


def test_pair_force_rotation_and_periodic_image():
    """Same pair rotated to a random direction and split across a periodic face:
    the force is the closed-form magnitude along e = r_ij / r."""
    rng = np.random.default_rng(3)
    for _ in range(20):
        e = rng.standard_normal(3); e /= np.linalg.norm(e)
        r = rng.uniform(0.05, 0.99)
        vr = rng.standard_normal(3)
        xj = np.array([0.01, 5.99, 3.0])
        xi_ = np.mod(xj + r * e, 6.0)
        sy = _pair_system(xi_, xj, vr, [0, 0, 0], sigma=0.0)
        f, _, _ = oracle.forces(sy, sy.x, sy.v, sy.tag, sy.type, 3)
        wC = 1 - r
        mag = 25.0 * wC - 4.5 * wC * np.dot(e, vr)
        np.testing.assert_allclose(f[:, 0], mag * e, rtol=1e-9, atol=1e-11)
        np.testing.assert_array_equal(f[:, 1], -f[:, 0])   # Newton's third law, bitwise


def test_dissipative_vanishes_for_perpendicular_velocity_and_outside_cutoff():
    sy = _pair_system([3.4, 3.0, 3.0], [3.0, 3.0, 3.0], [0.0, 2.0, -1.0], [0.0, 0.0, 0.0],
                      a=0.0, sigma=0.0)
    f, _, _ = oracle.forces(sy, sy.x, sy.v, sy.tag, sy.type, 1)
    np.testing.assert_allclose(f, 0.0, atol=1e-15)
    sy = _pair_system([4.0 + 1e-9, 3.0, 3.0], [3.0, 3.0, 3.0], [1.0, 0.0, 0.0], [0, 0, 0])
    f, _, npair = oracle.forces(sy, sy.x, sy.v, sy.tag, sy.type, 1)
    np.testing.assert_array_equal(f, 0.0)
    assert npair.sum() == 0


def test_type_pair_table_lookup():
    """a_ij comes from the (type_i, type_j) entry of the symmetric table."""
    a = np.array([[25.0, 75.0, 35.0], [75.0, 25.0, 75.0], [35.0, 75.0, 25.0]])
    x = np.array([[3.0, 3.0, 3.0], [3.5, 3.0, 3.0]]).T.copy()
    for t0, t1 in [(0, 1), (1, 2), (0, 2), (2, 2)]:
        sy = di.System(box=np.array([6.0] * 3), x=x, v=np.zeros((3, 2)),
                       tag=np.array([0, 1], dtype=np.uint32), type=np.array([t0, t1], dtype=np.uint8),
                       n_types=3, a=a, gamma=np.zeros((3, 3)), sigma=np.zeros((3, 3)))
        f, _, _ = oracle.forces(sy, sy.x, sy.v, sy.tag, sy.type, 1)
        np.testing.assert_allclose(f[0, 0], -a[t0, t1] * 0.5, rtol=1e-15)


def test_bond_and_body_force():
    """Harmonic bond -k (r - r0) e (Sec. 4.5) and the +/- g body force (Sec. 4.2)."""
    x = np.array([[1.0, 1.0, 1.0], [1.9, 1.0, 1.0], [3.0, 3.0, 3.0]]).T.copy()
    partner = np.array([[-1, 1], [0, -1], [-1, -1]], dtype=np.int32)
    sy = di.System(box=np.array([5.0, 6.0, 5.0]), x=x, v=np.zeros((3, 3)),
                   tag=np.arange(3, dtype=np.uint32), type=np.zeros(3, dtype=np.uint8),
                   a=np.array([[0.0]]), gamma=np.array([[0.0]]), sigma=np.array([[0.0]]),
                   bond_k=100.0, bond_r0=0.7, partner=partner, body_g=0.055, body_split=3.0)
    f, pe, _ = oracle.forces(sy, sy.x, sy.v, sy.tag, sy.type, 1)
    # r_01 = -0.9 along x: F_0 = -k (0.9 - 0.7) * (-1) = +20 ; plus body +g (y = 1 < 3)
    np.testing.assert_allclose(f[:, 0], [20.0 + 0.055, 0, 0], rtol=1e-12)
    np.testing.assert_allclose(f[:, 1], [-20.0 + 0.055, 0, 0], rtol=1e-12)
    np.testing.assert_allclose(f[:, 2], [-0.055, 0, 0], rtol=0, atol=0)   # y = 3 is not < 3
    sy.x[1, 2] = 2.999
    f, _, _ = oracle.forces(sy, sy.x, sy.v, sy.tag, sy.type, 1)
    np.testing.assert_allclose(f[0, 2], 0.055)
    np.testing.assert_allclose(pe[:2].sum(), 0.5 * 100 * 0.2**2, rtol=1e-12)


def test_forces_superpose_pairwise():
    """Eq (2): f_i is the plain sum of pair forces; check against pair-by-pair calls."""
    s = di.uniform_fluid(40, (3.2, 3.1, 3.3), 8)
    f, _, _ = oracle.forces(s, s.x, s.v, s.tag, s.type, 5)
    rng = np.random.default_rng(0)
    for i in rng.choice(40, 5, replace=False):
        tot = np.zeros(3)
        for j in range(40):
            if j == i:
                continue
            sub = di.System(**{**s.__dict__})
            sub.x = s.x[:, [i, j]].copy(); sub.v = s.v[:, [i, j]].copy()
            sub.tag = s.tag[[i, j]].copy(); sub.type = s.type[[i, j]].copy()
            fij, _, _ = oracle.forces(sub, sub.x, sub.v, sub.tag, sub.type, 5)
            tot += fij[:, 0]
        np.testing.assert_allclose(f[:, i], tot, rtol=1e-12, atol=1e-12)


# ----------------------------------------------------- neighbour sets ----

def _csr_sets(off, idx):
    return [set(idx[off[i]:off[i + 1]].tolist()) for i in range(len(off) - 1)]


@pytest.mark.parametrize("maker", [
    lambda: di.small_fluid(1),
    lambda: di.edge_case_fluid(),
    lambda: di.uniform_fluid(900, (7.3, 5.2, 8.9), 4),
    lambda: di.poiseuille(box=(6.0, 12.0, 4.0)),
])
def test_neighbors_brute_equals_cells(maker):
    s = maker()
    o1, i1 = oracle.neighbors(s.x, s.box, 1.0, mode="brute")
    o2, i2 = oracle.neighbors(s.x, s.box, 1.0, mode="cells")
    np.testing.assert_array_equal(o1, o2)
    np.testing.assert_array_equal(i1, i2)
    for i in range(s.n):
        row = i1[o1[i]:o1[i + 1]]
        assert np.all(np.diff(row) > 0)          # strictly ascending (Sec. 3.3.2)
        assert i not in row                      # no self pair
    sets = _csr_sets(o1, i1)
    for i, row in enumerate(sets):               # symmetric relation
        for j in row:
            assert i in sets[j]


def test_neighbors_match_kdtree_away_from_ties():
    """Independent periodic k-d tree (scipy) agrees on every pair whose
    distance is not within 1e-9 of r_list (where <= vs < and rounding differ)."""
    from scipy.spatial import cKDTree
    s = di.uniform_fluid(2000, (9.5, 8.25, 7.75), 21)
    off, idx = oracle.neighbors(s.x, s.box, 1.0)
    pts = s.x.T.copy()
    tree = cKDTree(pts, boxsize=s.box)
    pairs = tree.query_pairs(1.0 + 1e-9, output_type="ndarray")
    inner = tree.query_pairs(1.0 - 1e-9, output_type="ndarray")
    mine = {(i, j) for i in range(s.n) for j in idx[off[i]:off[i + 1]] if i < j}
    outer_set = {tuple(p) for p in pairs}
    inner_set = {tuple(p) for p in inner}
    assert inner_set <= mine <= outer_set
    assert len(outer_set - inner_set) < 5


def test_neighbors_edge_cases_planted():
    s = di.edge_case_fluid()
    off, idx = oracle.neighbors(s.x, s.box, 1.0)
    row = lambda i: set(idx[off[i]:off[i + 1]].tolist())
    assert 3 not in row(2)          # exactly r_c: excluded (strict test)
    assert 5 in row(4)              # one ulp inside r_c: included
    assert 7 not in row(6)          # one ulp outside
    assert 11 in row(10)            # through the periodic x face (0.4 apart)
    assert 1 in row(0)              # (0,0,0) and (L-ulp)^3 are ~ulp apart through the corner


# ------------------------------------------------------- cells / reorder --

def test_cell_grid_margin_rule():
    np.testing.assert_array_equal(oracle.cell_grid([10.0, 10.0, 10.0], 1.0), [9, 9, 9])
    np.testing.assert_array_equal(oracle.cell_grid([10.5, 3.5, 174.716], 1.0), [10, 3, 174])
    with pytest.raises(ValueError):
        oracle.cell_grid([3.0, 5.0, 5.0], 1.0)


def test_morton_rank_power_of_two_is_the_code():
    """On a 2^k grid every Morton code is used, so rank == code (closed form)."""
    nc = np.array([8, 8, 8], dtype=np.int32)
    rank = oracle.morton_rank_table(nc)
    for c in range(512):
        cx, cy, cz = c % 8, (c // 8) % 8, c // 64
        code = 0
        for b in range(3):
            code |= ((cx >> b) & 1) << (3 * b)
            code |= ((cy >> b) & 1) << (3 * b + 1)
            code |= ((cz >> b) & 1) << (3 * b + 2)
        assert rank[c] == code


def _zorder_less(a, b):
    """Z-order comparison without building codes: compare the coordinate whose
    highest differing bit is the largest, ties broken z > y > x."""
    best_dim, best_msb = -1, -1
    for d in (2, 1, 0):                      # z, y, x: z wins ties of equal msb
        diff = a[d] ^ b[d]
        msb = diff.bit_length() - 1
        if msb > best_msb:
            best_dim, best_msb = d, msb
    if best_dim < 0:
        return False
    return a[best_dim] < b[best_dim]


def test_morton_rank_general_grid_by_comparison():
    nc = np.array([5, 3, 6], dtype=np.int32)
    rank = oracle.morton_rank_table(nc)
    cells = [(c % 5, (c // 5) % 3, c // 15) for c in range(90)]
    assert sorted(rank.tolist()) == list(range(90))
    order = sorted(range(90), key=lambda c: rank[c])
    for p, q in zip(order[:-1], order[1:]):
        assert _zorder_less(cells[p], cells[q])


def test_reorder_permutation_definition():
    s = di.shuffled(di.small_fluid(2), 77)
    perm, cs = oracle.reorder(s.x, s.tag, s.box, 1.0)
    nc = oracle.cell_grid(s.box, 1.0)
    rank = oracle.morton_rank_table(nc)
    inv = nc / s.box
    c = np.minimum(nc[:, None] - 1, (s.x * inv[:, None]).astype(np.int64))
    lin = c[0] + nc[0] * (c[1] + nc[1] * c[2])
    r = rank[lin]
    ref = np.lexsort((s.tag, r))                   # primary: rank, secondary: tag
    np.testing.assert_array_equal(perm, ref)
    assert cs[0] == 0 and cs[-1] == s.n
    counts = np.bincount(r, minlength=len(cs) - 1)
    np.testing.assert_array_equal(np.diff(cs), counts)


# ------------------------------------------------ integrator invariants --

def test_ballistic_motion():
    """a = gamma = sigma = 0: x_n = x_0 + n dt v_0 (mod L), v unchanged."""
    s = di.uniform_fluid(300, (5.0, 5.0, 5.0), 13, a=0.0, gamma=0.0, sigma=0.0)
    f0, _, _ = oracle.forces(s, s.x, s.v, s.tag, s.type, 0)
    assert np.all(f0 == 0)
    x, v, f, red, _ = oracle.run(s, s.x, s.v, f0, s.tag, s.type, 0, 50)
    np.testing.assert_array_equal(v, s.v)
    expect = np.mod(s.x + 50 * s.dt * s.v, s.box[:, None])
    d = np.abs(x - expect)
    d = np.minimum(d, s.box[:, None] - d)
    assert d.max() < 1e-12


def test_harmonic_dimer_period():
    """Bond-only dimer (m = 1): relative coordinate oscillates with period
    2 pi / sqrt(2k); energy error stays O(dt^2)."""
    k, r0 = 100.0, 0.7
    x = np.array([[2.0, 2.0, 2.0], [2.9, 2.0, 2.0]]).T.copy()
    partner = np.array([[-1, 1], [0, -1]], dtype=np.int32)
    s = di.System(box=np.array([4.0, 4.0, 4.0]), x=x, v=np.zeros((3, 2)),
                  tag=np.arange(2, dtype=np.uint32), type=np.zeros(2, dtype=np.uint8),
                  a=np.array([[0.0]]), gamma=np.array([[0.0]]), sigma=np.array([[0.0]]),
                  bond_k=k, bond_r0=r0, partner=partner, dt=0.001)
    f0, _, _ = oracle.forces(s, s.x, s.v, s.tag, s.type, 0)
    xx, vv, ff = s.x, s.v, f0
    seps, energies = [], []
    for _ in range(2000):
        xx, vv, ff, red, _ = oracle.run(s, xx, vv, ff, s.tag, s.type, 0, 1)
        sep = xx[0, 1] - xx[0, 0]
        seps.append(sep - r0)
        energies.append(0.5 * np.sum(vv**2) + 0.5 * k * (abs(sep) - r0) ** 2)
    seps = np.array(seps)
    t = (np.arange(len(seps)) + 1) * s.dt
    up = np.where((seps[:-1] < 0) & (seps[1:] >= 0))[0]
    tc = t[up] + s.dt * (-seps[up]) / (seps[up + 1] - seps[up])
    period = np.mean(np.diff(tc))
    np.testing.assert_allclose(period, 2 * np.pi / np.sqrt(2 * k), rtol=2e-3)
    e = np.array(energies)
    assert (e.max() - e.min()) / e.mean() < 5e-3


def test_momentum_conserved_by_pair_forces():
    """Newton's third law: total pair + bond force is zero to round-off."""
    s = di.amphiphile(n=4000, seed=12)
    f, _, _ = oracle.forces(s, s.x, s.v, s.tag, s.type, 3, mode="cells")
    scale = np.abs(f).sum()
    assert np.abs(f.sum(axis=1)).max() < 1e-14 * scale
    # and over many steps the total momentum stays at round-off
    x, v, f2, red, _ = oracle.run(s, s.x, s.v, f, s.tag, s.type, 0, 20)
    assert np.abs(red[:, :3]).max() < 1e-10


def test_conservative_fluid_energy_bounded():
    """gamma = sigma = 0: velocity Verlet is symplectic; total energy stays
    within O(dt^2) of its start over 400 steps (no drift)."""
    s = di.uniform_fluid(375, (5.0, 5.0, 5.0), 31, gamma=0.0, sigma=0.0, dt=0.005)
    f, pe, _ = oracle.forces(s, s.x, s.v, s.tag, s.type, 0)
    e0 = 0.5 * np.sum(s.v**2) + pe.sum()
    x, v, f, red, _ = oracle.run(s, s.x, s.v, f, s.tag, s.type, 0, 400)
    e = 0.5 * red[:, 3] + red[:, 4]
    assert np.abs(e - e0).max() / abs(e0) < 2e-3


@pytest.mark.slow
def test_kbt_fluctuation_dissipation():
    """Eq (9): equilibrium k_BT = sigma^2 / (2 gamma) = 1, over 3(N-1) degrees
    of freedom, within 3 sigma of block statistics plus a time-step bias allowance."""
    s = di.uniform_fluid(375, (5.0, 5.0, 5.0), 41)
    f, _, _ = oracle.forces(s, s.x, s.v, s.tag, s.type, 0)
    x, v, f, red, _ = oracle.run(s, s.x, s.v, f, s.tag, s.type, 0, 1000)
    x, v, f, red, _ = oracle.run(s, x, v, f, s.tag, s.type, 1000, 12000)
    kbt = red[:, 6]
    blocks = kbt.reshape(40, -1).mean(axis=1)
    err = blocks.std(ddof=1) / np.sqrt(len(blocks))
    assert abs(kbt.mean() - 1.0) < 3 * err + 0.02, (kbt.mean(), err)
    # a different sigma/gamma ratio moves k_BT accordingly
    s2 = di.uniform_fluid(375, (5.0, 5.0, 5.0), 42, gamma=4.5, sigma=np.sqrt(2 * 4.5 * 0.5))
    f, _, _ = oracle.forces(s2, s2.x, s2.v, s2.tag, s2.type, 0)
    x, v, f, red, _ = oracle.run(s2, s2.x, s2.v, f, s2.tag, s2.type, 0, 6000)
    np.testing.assert_allclose(red[2000:, 6].mean(), 0.5, rtol=0.04)


@pytest.mark.slow
def test_reverse_poiseuille_parabola():
    """Steady reverse-Poiseuille flow: each channel's mean v_x(y) is the
    parabola F d^2/(8 nu) (1 - (2z/d)^2) of Eq (10)'s steady part, with zero
    velocity on the planes where the body force flips."""
    g = 0.1
    s = di.poiseuille(seed=5, box=(8.0, 12.0, 4.0), rho=3.0, g=g)
    f, _, _ = oracle.forces(s, s.x, s.v, s.tag, s.type, 0)
    nb = 24
    x, v, f, red, prof = oracle.run(s, s.x, s.v, f, s.tag, s.type, 0, 4000,
                                    profile=(1, 0, nb, 1000))
    y = (np.arange(nb) + 0.5) * s.box[1] / nb
    d = s.box[1] / 2
    fits = []
    for lo, sign in ((0.0, 1.0), (d, -1.0)):
        m = (y > lo) & (y < lo + d)
        z = y[m] - (lo + d / 2)
        basis = 1 - (2 * z / d) ** 2
        amp = np.dot(basis, prof[m]) / np.dot(basis, basis)
        resid = prof[m] - amp * basis
        fits.append(sign * amp)
        assert sign * amp > 0
        assert np.sqrt(np.mean(resid**2)) < 0.08 * abs(amp), (amp, resid)
        # free quadratic: linear term ~ 0, curvature matches the parabola
        c2, c1, c0 = np.polyfit(z, prof[m], 2)
        assert abs(c1) < 0.05 * abs(amp)
    np.testing.assert_allclose(fits[0], fits[1], rtol=0.1)
    nu = g * d * d / (8 * np.mean(fits))
    assert 0.2 < nu < 1.5                       # a DPD-fluid kinematic viscosity


# ------------------------------------------------------------ VJP pins --

def _vjp_fd_check(s, step, h, rtol, rng):
    nbr = oracle.neighbors(s.x, s.box, 1.0)
    g = rng.standard_normal(s.x.shape)
    xb, vb, ab, gb = oracle.forces_vjp(s, s.x, s.v, s.tag, s.type, step, g, nbr=nbr)

    def loss(x=None, v=None, a=None, gamma=None):
        sy = di.System(**{**s.__dict__})
        if a is not None:
            sy.a = a
        if gamma is not None:
            sy.gamma = gamma
        f, _, _ = oracle.forces(sy, s.x if x is None else x, s.v if v is None else v,
                                s.tag, s.type, step, nbr=nbr)
        return np.sum(f * g)

    for _ in range(3):
        dx = rng.standard_normal(s.x.shape)
        fd = (loss(x=s.x + h * dx) - loss(x=s.x - h * dx)) / (2 * h)
        np.testing.assert_allclose(np.sum(xb * dx), fd, rtol=rtol)
        dv = rng.standard_normal(s.x.shape)
        fd = (loss(v=s.v + h * dv) - loss(v=s.v - h * dv)) / (2 * h)
        np.testing.assert_allclose(np.sum(vb * dv), fd, rtol=rtol)
    nt = s.n_types
    for t in range(nt):
        for u in range(t, nt):
            da = np.zeros((nt, nt)); da[t, u] = da[u, t] = 1.0
            fd = (loss(a=s.a + h * da) - loss(a=s.a - h * da)) / (2 * h)
            np.testing.assert_allclose(ab[t, u], fd, rtol=rtol, atol=1e-7)
            np.testing.assert_allclose(ab[u, t], ab[t, u])
            fd = (loss(gamma=s.gamma + h * da) - loss(gamma=s.gamma - h * da)) / (2 * h)
            np.testing.assert_allclose(gb[t, u], fd, rtol=rtol, atol=1e-7)


def test_forces_vjp_finite_differences_s1():
    rng = np.random.default_rng(1)
    s = di.uniform_fluid(200, (4.0, 4.0, 4.0), 17, s=1.0)
    s.type = rng.integers(0, 2, s.n).astype(np.uint8)
    s.n_types = 2
    s.a = np.array([[25.0, 40.0], [40.0, 25.0]])
    s.gamma = np.array([[4.5, 3.0], [3.0, 4.5]])
    s.sigma = np.full((2, 2), 3.0)
    _vjp_fd_check(s, 9, 1e-6, 1e-6, rng)


def test_forces_vjp_finite_differences_s_half_with_bonds():
    rng = np.random.default_rng(2)
    s = di.amphiphile(n=400, seed=19, chain_fraction=0.2)
    # small h: for s = 1/2 the weight derivative (1 - r)^(-1/2) is steep near r_c
    _vjp_fd_check(s, 4, 1e-7, 1e-5, rng)


# ------------------------------------------------- trajectory adjoint --

@pytest.mark.parametrize("s_exp,h,rtol", [(1.0, 1e-6, 1e-7), (0.5, 1e-7, 2e-6)])
def test_force_matching_gradient_finite_differences(s_exp, h, rtol):
    """The oracle's reverse sweep of the velocity-Verlet trajectory equals
    central finite differences of its own loss, for a_AB, gamma and random
    directions in x0 and v0.  With s = 1/2 the weight's derivative diverges
    at r_c, so pairs near the cutoff need a smaller h for the difference
    quotient to converge (its error shrinks with h: ~1e-3 at h = 1e-5,
    ~2e-7 at h = 1e-7)."""
    s = di.binary_mixture(n=300, box=(5.0, 5.0, 4.0), seed=21, a_ab=40.0)
    s.s = s_exp
    K = 6
    rng = np.random.default_rng(4)
    ref = oracle.trajectory(s, s.x, s.v, K, a=np.array([[25.0, 31.0], [31.0, 25.0]]))
    T = np.stack([ref[k][2] for k in range(1, K + 1)])
    L, ga, gg, gx, gv = oracle.force_matching_grad(s, s.x, s.v, K, T)

    def loss(a=None, gamma=None, x=None, v=None):
        tr = oracle.trajectory(s, s.x if x is None else x, s.v if v is None else v, K, a=a, gamma=gamma)
        return sum(float(np.sum((tr[k][2] - T[k - 1]) ** 2)) for k in range(1, K + 1))

    np.testing.assert_allclose(loss(), L, rtol=1e-13)
    da = np.array([[0.0, 1.0], [1.0, 0.0]])
    fd = (loss(a=s.a + h * da) - loss(a=s.a - h * da)) / (2 * h)
    np.testing.assert_allclose(ga[0, 1], fd, rtol=rtol)
    assert ga[0, 1] == ga[1, 0]
    for t, u in ((0, 0), (0, 1)):
        dg = np.zeros((2, 2)); dg[t, u] = dg[u, t] = 1.0
        fd = (loss(gamma=s.gamma + h * dg) - loss(gamma=s.gamma - h * dg)) / (2 * h)
        np.testing.assert_allclose(gg[t, u], fd, rtol=rtol)
    dx = rng.standard_normal(s.x.shape)
    fd = (loss(x=s.x + h * dx) - loss(x=s.x - h * dx)) / (2 * h)
    np.testing.assert_allclose(np.sum(gx * dx), fd, rtol=rtol)
    dv = rng.standard_normal(s.v.shape)
    fd = (loss(v=s.v + h * dv) - loss(v=s.v - h * dv)) / (2 * h)
    np.testing.assert_allclose(np.sum(gv * dv), fd, rtol=rtol)


# ------------------------------------------------ border exchange (Alg 6) --

@pytest.mark.parametrize("box,n,width", [((7.0, 6.0, 8.0), 1000, 1.0), ((5.0, 9.5, 6.25), 900, 1.3)])
def test_staged_halo_reproduces_periodic_neighbours(box, n, width):
    """The border lists and ghost records of the three-stage exchange on one
    brick spanning the periodic box (x faces, then y faces over owned + x
    ghosts, then z faces over all): every periodic neighbour pair of an
    owned particle (scipy's periodic k-d tree) appears exactly once among
    the owned + ghost particles at plain Euclidean distance (a non-periodic
    k-d tree), and no other pair does.  A wrong band side, a wrong shift
    sign or a missing stage loses or duplicates pairs."""
    from scipy.spatial import cKDTree
    s = di.uniform_fluid(n, box, 77)
    X, V, T, Y, stages = oracle.staged_halo(s.x, s.v, s.tag, s.type, s.box, width)
    assert X.shape[1] > n
    # positions of the ghosts lie within `width` outside the box, no farther
    lo = -width * np.ones(3)[:, None]
    hi = np.asarray(box)[:, None] + width
    assert np.all(X >= lo - 1e-12) and np.all(X < hi + 1e-12)
    per = cKDTree(s.x.T, boxsize=np.asarray(box))
    flat = cKDTree(X.T)
    r = width * (1.0 - 1e-9)          # away from pairs at the radius itself
    for i in range(n):
        want = sorted(s.tag[j] for j in per.query_ball_point(s.x[:, i], r) if j != i)
        got = sorted(T[j] for j in flat.query_ball_point(X[:, i], r) if j != i)
        assert got == want, i
    # the velocities and types travel with the copies (tags are the
    # original indices here)
    np.testing.assert_array_equal(V, s.v[:, T])
    np.testing.assert_array_equal(Y, s.type[T])
    for d, (off, idx) in enumerate(stages):
        assert np.all(np.diff(off) >= 0)
        for f in range(6):
            seg = idx[off[f]:off[f + 1]]
            assert np.all(np.diff(seg) > 0)                 # ascending
            if f // 2 != d:
                assert seg.size == 0                        # only this stage's faces


def test_border_lists_band_edges():
    """Planted positions on the band edges of a sub-brick: a particle exactly
    at lo + width is not sent through the low face, one exactly at
    hi - width is sent through the high face, and a particle outside the
    brick on the low side is sent through the low face only."""
    lo = np.array([1.0, 2.0, 3.0])
    hi = np.array([5.0, 6.5, 7.25])
    w = 0.75
    x = np.array([[lo[0] + w, hi[0] - w, lo[0] + w - 2 ** -40, 0.5, 3.0],
                  [4.0, 4.0, 4.0, 4.0, hi[1] - w],
                  [5.0, 5.0, 5.0, 5.0, 5.0]])
    off, idx = oracle.border_lists(x, lo, hi, w)
    lists = [list(idx[off[f]:off[f + 1]]) for f in range(6)]
    assert lists[0] == [2, 3]
    assert lists[1] == [1]
    assert lists[2] == []
    assert lists[3] == [4]
    assert lists[4] == [] and lists[5] == []
    off_x, idx_x = oracle.border_lists(x, lo, hi, w, face_mask=0b000010)
    assert list(off_x) == [0, 0, 1, 1, 1, 1, 1] and list(idx_x) == [1]


# ------------------------------------------- TEA generator (A/B study) --

def _tea_decipher(rounds, v, k):
    """TEA's inverse, written from the cipher's definition: the cycles
    undone in reverse order (second half first, the sum counting down)."""
    m = 0xFFFFFFFF
    delta = 0x9E3779B9
    y, z = int(v[0]), int(v[1])
    s = (delta * rounds) & m
    for _ in range(rounds):
        z = (z - ((((y << 4) & m) + k[2]) ^ ((y + s) & m) ^ ((y >> 5) + k[3]))) & m
        y = (y - ((((z << 4) & m) + k[0]) ^ ((z + s) & m) ^ ((z >> 5) + k[1]))) & m
        s = (s - delta) & m
    return y, z


@pytest.mark.parametrize("rounds", [1, 4, 16, 32])
def test_tea_inverts_and_diffuses(rounds):
    rng = np.random.default_rng(rounds)
    flips = []
    for _ in range(300):
        v = rng.integers(0, 2 ** 32, size=2, dtype=np.uint64).astype(np.uint32)
        k = [int(t) for t in rng.integers(0, 2 ** 32, size=4, dtype=np.uint64)]
        w = oracle.tea(rounds, v, np.array(k, dtype=np.uint32))
        assert _tea_decipher(rounds, w, k) == (int(v[0]), int(v[1]))
        bit = int(rng.integers(0, 64))
        v2 = v.copy()
        v2[bit // 32] ^= np.uint32(1 << (bit % 32))
        w2 = oracle.tea(rounds, v2, np.array(k, dtype=np.uint32))
        flips.append(bin(int(w[0] ^ w2[0])).count("1") + bin(int(w[1] ^ w2[1])).count("1"))
    if rounds >= 4:
        assert 28 < np.mean(flips) < 36          # half of the 64 output bits


def test_tea_signature_inputs():
    for t in (0, 1, 7, 0x80000000, 0x12345678, 0xFFFFFFFF):
        rev = int(format(t, "032b")[::-1], 2)
        assert oracle.tea_sig_inputs(t, 0.0, 0.0, 0.0)[0] == rev
    # leading mantissa bits: 1.5 = 1.1b (top bit), 1.25 = 1.01b; bit b of
    # x, y, z goes to 3b, 3b + 1, 3b + 2; bit 10 of z (position 32) is dropped
    assert oracle.tea_sig_inputs(0, 1.5, 1.0, 1.0)[1] == 1 << 30
    assert oracle.tea_sig_inputs(0, 1.0, 1.5, 1.0)[1] == 1 << 31
    assert oracle.tea_sig_inputs(0, 1.0, 1.0, 1.5)[1] == 0
    assert oracle.tea_sig_inputs(0, 1.0, -1.25, 1.0)[1] == 1 << 28
    assert oracle.tea_sig_inputs(0, 1.0 + 2.0 ** -52, 1.0, 1.0)[1] == 0      # below the 11 bits
    assert oracle.tea_sig_inputs(0, 1.0 + 2.0 ** -11, 1.0, 1.0)[1] == 1      # the 11th bit


def test_tea_pair_gaussians_moments_and_symmetry():
    """The paper checks this generator by the moments of its output (up to
    the fourth); over 2^20 pairs of random signatures: 0, 1, 0, 3 within a
    few standard errors, symmetric in the pair, and each pair's words give
    the Box-Muller value recomputed with numpy."""
    rng = np.random.default_rng(5)
    n = 1 << 20
    si = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    sj = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    w, xi = oracle.tea_xi(si, sj, 17, 99)
    w2, xi2 = oracle.tea_xi(sj, si, 17, 99)
    np.testing.assert_array_equal(xi, xi2)
    se = 1.0 / np.sqrt(n)
    assert abs(xi.mean()) < 5 * se
    assert abs(np.mean(xi ** 2) - 1.0) < 5 * np.sqrt(2.0) * se
    assert abs(np.mean(xi ** 3)) < 5 * np.sqrt(15.0) * se
    assert abs(np.mean(xi ** 4) - 3.0) < 5 * np.sqrt(96.0) * se
    u1 = (w[:, 0].astype(np.float64) + 0.5) / 2.0 ** 32
    u2 = w[:, 1].astype(np.float64) / 2.0 ** 32
    np.testing.assert_allclose(xi, np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2), rtol=0, atol=1e-13)
    # Step to step, the values decorrelate through the signatures (rehashed
    # with the step in the key, 16 cycles); four cycles alone do not
    # decorrelate a key that changes by one: with the signatures held fixed
    # the next step's values correlate strongly.
    _, xi_frozen = oracle.tea_xi(si, sj, 18, 99)
    assert np.corrcoef(xi, xi_frozen)[0, 1] > 0.3
    m = 1 << 16
    tags = rng.permutation(m).astype(np.uint32)
    vel = rng.standard_normal((3, m))
    a, b = rng.integers(0, m, size=n), rng.integers(0, m, size=n)
    s17 = oracle.tea_signatures(tags, vel, 17, 99)
    s18 = oracle.tea_signatures(tags, vel, 18, 99)
    _, x17 = oracle.tea_xi(s17[a], s17[b], 17, 99)
    _, x18 = oracle.tea_xi(s18[a], s18[b], 18, 99)
    assert abs(np.corrcoef(x17, x18)[0, 1]) < 5 * se
