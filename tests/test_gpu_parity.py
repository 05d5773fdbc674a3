"""GPU (libdpd) against the CPU oracle, element by element.

Bars: reorder permutations and neighbour sets bit-exact; FP64 forces within
1e-12 of the per-particle summation scale S_i = sum of the magnitudes of the
added terms (and 1e-12 globally in L2); the mixed form within 1e-5 of |F| in
the global L2 norm (and its 99.99th percentile per particle).  Positions
after a step are bit-exact given the same forces.
"""
import numpy as np
import pytest

import dpd_inputs as di
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_1311_0402_amd")

FP64_TOL = 1e-12
MIXED_TOL = 1e-5


def _device_state(s):
    st = P.State.empty(s.n)
    st.x.copy_(torch.as_tensor(s.x))
    st.v.copy_(torch.as_tensor(s.v))
    st.tag.copy_(torch.as_tensor(s.tag.view(np.int32)))
    st.type.copy_(torch.as_tensor(s.type))
    return st


def _sorted_system(s, precision=P.FP64, capacity=None):
    params = P.Params.like(s)
    sim = P.System(params, s.n, precision, capacity=capacity)
    sim.load(s.x, s.v, s.tag, s.type, step=0)
    torch.cuda.synchronize()
    return sim


def _check_fp64(f_gpu, f_ref, scale):
    d = np.linalg.norm(f_gpu - f_ref, axis=0)
    bound = FP64_TOL * np.maximum(scale, 1e-300)
    bad = np.nonzero(d > bound)[0]
    assert bad.size == 0, f"{bad.size} particles over 1e-12 S_i, worst ratio {np.max(d / bound):.3g}"
    assert np.linalg.norm(f_gpu - f_ref) <= FP64_TOL * np.linalg.norm(f_ref)


def _systems():
    return {
        "fluid3000": di.shuffled(di.small_fluid(1), 3),
        "edge": di.edge_case_fluid(),
        "ragged": di.uniform_fluid(2717, (9.3, 7.6, 12.9), 8),
        "amphiphile": di.amphiphile(n=6000, seed=4),
        "poiseuille": di.poiseuille(seed=9, box=(6.0, 12.0, 5.0), rho=4.0),
        "clustered": di.clustered_fluid(),
        # the tile list builder: partial tiles at the high faces, the planted
        # cases, and a cluster whose tile neighbourhood overflows the LDS
        # staging; grids narrower than a tile's 10 x 6 x 6-cell neighbourhood
        # (cells staged once per periodic image), down to 3 cells a side
        "tiny_tiles": di.uniform_fluid(110, (3.3, 3.4, 3.6), 21),
        "thin_tiles": di.uniform_fluid(700, (3.1, 12.5, 5.4), 22),
        "slab_tiles": di.uniform_fluid(1500, (14.2, 4.3, 7.7), 23),
        "ragged_tiles": di.uniform_fluid(5000, (13.7, 11.1, 9.3), 11),
        "edge_tiles": di.edge_case_fluid(seed=12, box=(12.0, 10.5, 6.5), n=800),
        "clustered_tiles": di.clustered_fluid(seed=13, box=(12.0, 10.5, 7.0), n_cluster=1600, n_rest=800,
                                              size=1.5),
        # a blob whose rows outgrow the slab width inside a tile the tile
        # builder walks (the build then falls back to the direct pass)
        "blob_tiles": di.clustered_fluid(seed=14, box=(12.0, 10.5, 7.0), n_cluster=300, n_rest=1500, size=2.0),
    }


# ---------------------------------------------------------------- reorder --

@pytest.mark.parametrize("name", list(_systems()))
def test_bin_reorder_bitexact(name):
    s = _systems()[name]
    params = P.Params.like(s)
    nc = P.cell_grid(params)
    np.testing.assert_array_equal(nc, oracle.cell_grid(s.box, s.r_c))
    src = _device_state(s)
    dst = P.State.empty(s.n)
    cells = P.Cells.empty(s.n, int(np.prod(nc)))
    ws = P.alloc_workspace(params, s.n)
    x32 = torch.empty((s.n, 4), dtype=torch.float32, device="cuda")
    v32 = torch.empty_like(x32)
    P.dpd_bin_reorder(params, src, dst, cells, ws, x32=x32, v32=v32)
    torch.cuda.synchronize()
    perm_ref, cs_ref = oracle.reorder(s.x, s.tag, s.box, s.r_c)
    perm = cells.perm.cpu().numpy()
    np.testing.assert_array_equal(perm, perm_ref)
    np.testing.assert_array_equal(cells.cell_start.cpu().numpy(), cs_ref)
    np.testing.assert_array_equal(dst.x.cpu().numpy(), s.x[:, perm_ref])
    np.testing.assert_array_equal(dst.v.cpu().numpy(), s.v[:, perm_ref])
    np.testing.assert_array_equal(dst.tag.cpu().numpy().view(np.uint32), s.tag[perm_ref])
    np.testing.assert_array_equal(dst.type.cpu().numpy(), s.type[perm_ref])
    iot = cells.idx_of_tag.cpu().numpy()
    np.testing.assert_array_equal(iot[s.tag[perm_ref]], np.arange(s.n))
    # packed FP32 copies: (offset inside the cell, tag bits), (velocity, type)
    cxyz = cells.cell_xyz.cpu().numpy().view(np.uint32)
    cc = np.stack([cxyz & 1023, (cxyz >> 10) & 1023, cxyz >> 20]).astype(np.float64)
    np.testing.assert_array_equal(cc, np.minimum(np.array(nc)[:, None] - 1,
                                                 (s.x[:, perm_ref] * (np.array(nc) / s.box)[:, None]).astype(np.int64)))
    ell = s.box / np.array(nc)
    xs = s.x[:, perm_ref]
    xw = x32.cpu().numpy()
    vw = v32.cpu().numpy()
    np.testing.assert_array_equal(xw[:, :3].T, (xs - cc * ell[:, None]).astype(np.float32))
    np.testing.assert_array_equal(xw[:, 3].view(np.uint32), s.tag[perm_ref])
    np.testing.assert_array_equal(vw[:, :3].T, s.v[:, perm_ref].astype(np.float32))
    np.testing.assert_array_equal(vw[:, 3].view(np.uint32), s.type[perm_ref].astype(np.uint32))


def test_bin_reorder_is_deterministic_and_idempotent():
    s = di.shuffled(di.small_fluid(2), 5)
    sim = _sorted_system(s)
    x1, v1, _, t1, _ = sim.host_state()
    perm1 = sim.cells.perm.cpu().numpy()
    sim2 = _sorted_system(s)
    np.testing.assert_array_equal(sim2.cells.perm.cpu().numpy(), perm1)
    # reordering an already sorted state is the identity
    again = P.State.empty(s.n)
    P.dpd_bin_reorder(sim.params, sim.state, again, sim2.cells, sim.ws)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(sim2.cells.perm.cpu().numpy(), np.arange(s.n))


# ------------------------------------------------------------ neighbours --

@pytest.mark.parametrize("name", list(_systems()))
def test_neighbor_rows_bitexact(name):
    s = _systems()[name]
    sim = _sorted_system(s)
    x, _, _, _, _ = sim.host_state()
    off, idx = sim.host_nlist()
    off_ref, idx_ref = oracle.neighbors(x, s.box, s.r_c)
    np.testing.assert_array_equal(off, off_ref)
    np.testing.assert_array_equal(idx, idx_ref)      # same sets, same ascending order
    assert sim.check_status() == 0


def test_neighbor_overflow_flags_and_recovers():
    s = di.small_fluid(3)
    params = P.Params.like(s)
    sim = P.System(params, s.n, P.FP64, capacity=1000)
    src = _device_state(s)
    sim.reorder_from(src)
    sim.rebuild()
    torch.cuda.synchronize()
    st = int(sim.status.item())
    assert st & P._abi.STATUS_NLIST_OVERFLOW
    need = int(sim.nlist.offset[s.n].item())
    off_ref, idx_ref = oracle.neighbors(sim.host_state()[0], s.box, s.r_c)
    assert need == len(idx_ref)
    assert sim.fit_capacity()
    torch.cuda.synchronize()
    assert sim.check_status() == 0
    off, idx = sim.host_nlist()
    np.testing.assert_array_equal(idx, idx_ref)


# ---------------------------------------------------------------- forces --

@pytest.mark.parametrize("name", list(_systems()))
@pytest.mark.parametrize("step", [0, 7, (1 << 32) + 3])
def test_forces_fp64(name, step):
    s = _systems()[name]
    sim = _sorted_system(s)
    pe = torch.empty(s.n, dtype=torch.float64, device="cuda")
    sim.compute_forces(step, pe_out=pe)
    torch.cuda.synchronize()
    x, v, f, tag, typ = sim.host_state()
    f_ref, pe_ref, npair_ref, scale = oracle.forces(s, x, v, tag, typ, step, with_scale=True)
    _check_fp64(f, f_ref, scale)
    np.testing.assert_allclose(pe.cpu().numpy(), pe_ref, rtol=1e-12, atol=1e-12)
    stats = sim.stats.cpu().numpy()
    np.testing.assert_allclose(stats[0], pe_ref.sum(), rtol=1e-12)
    assert stats[1] == npair_ref.sum() / 2


@pytest.mark.parametrize("name", list(_systems()))
def test_forces_mixed(name):
    s = _systems()[name]
    sim = _sorted_system(s, precision=P.MIXED)
    x, v, f, tag, typ = sim.host_state()
    f_ref, _, _ = oracle.forces(s, x, v, tag, typ, 0)
    d = np.linalg.norm(f - f_ref, axis=0)
    rel = np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref)
    assert rel <= MIXED_TOL, rel
    rms = np.sqrt(np.mean(np.sum(f_ref**2, axis=0)))
    assert np.percentile(d / rms, 99.99) <= MIXED_TOL


def test_forces_antisymmetric_momentum():
    """Newton's third law on the device: sum of all forces ~ round-off."""
    s = di.amphiphile(n=6000, seed=8)
    sim = _sorted_system(s)
    _, _, f, _, _ = sim.host_state()
    assert np.abs(f.sum(axis=1)).max() < 1e-12 * np.abs(f).sum()


# ------------------------------------------------------------------ step --

def test_step_teacher_forced_100():
    """Each of 100 steps of the 3000-particle fluid against one oracle step
    from the GPU's own previous state: positions bit-exact, forces 1e-12 S_i."""
    s = di.small_fluid(1)
    sim = _sorted_system(s)
    red = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    prev = sim.host_state()
    for k in range(1, 101):
        sim.step(1, reductions=red)
        torch.cuda.synchronize()
        cur = sim.host_state()
        xo, vo, fo, red_ref = oracle.step(s, prev[0], prev[1], prev[2], prev[3], prev[4], k)
        o_prev = np.argsort(prev[3])
        o_cur = np.argsort(cur[3])
        np.testing.assert_array_equal(cur[0][:, o_cur], xo[:, o_prev], err_msg=f"step {k} x")
        # summation scale of this step's forces (velocity: the half-step one)
        vh = prev[1] + 0.5 * s.dt * prev[2]
        _, _, _, scale = oracle.forces(s, xo, vh, prev[3], prev[4], k, with_scale=True)
        _check_fp64(cur[2][:, o_cur], fo[:, o_prev], scale[o_prev])
        dv = np.abs(cur[1][:, o_cur] - vo[:, o_prev])
        assert np.all(dv <= 0.5 * s.dt * FP64_TOL * scale[o_prev] + 1e-15), f"step {k} v"
        r = red.cpu().numpy()[0]
        np.testing.assert_allclose(r[:3], red_ref[:3], atol=1e-9)
        np.testing.assert_allclose(r[3:7], red_ref[3:7], rtol=1e-12)
        prev = cur
    assert sim.step_count == 100
    assert sim.check_status() == 0


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_overflowing_rows_in_a_large_system(precision):
    """A dense blob (density ~50: rows of ~200 entries, beyond the slab's
    width) in a 700,000-particle fluid: the builder's slab is discarded and
    the direct pass, on its capped grid (more rows than its lanes, so a lane
    takes a second group), writes every row.  After a 2-step dpd_step call
    a seeded sample of rows, the blob's and the last ones included, equals
    the oracle's brute-force rows bit for bit, and their forces match."""
    side = (700_000 / 3.0) ** (1.0 / 3.0)
    s = di.clustered_fluid(seed=21, box=(side, side, side), n_cluster=400, n_rest=700_000, size=2.0)
    sim = _sorted_system(s, precision)
    sim.step(2)
    torch.cuda.synchronize()
    assert sim.check_status() == 0
    x, v, f, tag, typ = sim.host_state()
    off, idx = sim.host_nlist()
    assert np.diff(off).max() > 128
    blob = np.nonzero(tag < 400)[0]
    q = np.unique(np.concatenate([np.random.default_rng(5).choice(s.n, 600, replace=False), blob[:200],
                                  np.arange(s.n - 200, s.n)])).astype(np.int32)
    off_ref, idx_ref = oracle.neighbors(x, s.box, s.r_c, query=q)
    for k, i in enumerate(q):
        np.testing.assert_array_equal(idx[off[i]:off[i + 1]], idx_ref[off_ref[k]:off_ref[k + 1]],
                                      err_msg=f"row {i}")
    vh = v - 0.5 * s.dt * f
    f_ref, _, _, scale = oracle.forces(s, x, vh, tag, typ, 2, nbr=(off_ref, idx_ref), query=q, with_scale=True)
    if precision == P.FP64:
        _check_fp64(f[:, q], f_ref, scale)
    else:
        rel = np.linalg.norm(f[:, q] - f_ref) / np.linalg.norm(f_ref)
        assert rel <= MIXED_TOL, rel
    del sim
    torch.cuda.empty_cache()


@pytest.mark.parametrize("s_exp", [1.0, 2.0, 0.25])
@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_weight_exponents(s_exp, precision):
    """The weight w_R = (1 - r/r_c)^s of Eq (8) beyond s = 1/2: s = 1 and 2
    (the pass's own branches) and a general s = 1/4 (a power): the forces
    of the loaded state and of a 5-step call's final state against the
    oracle (FP64 within 1e-12 S_i, mixed within 1e-5 of |F|)."""
    s = di.uniform_fluid(3000, (10.0, 10.0, 10.0), 43, s=s_exp)
    sim = _sorted_system(s, precision)
    for k in (0, 5):
        if k:
            sim.step(k)
            torch.cuda.synchronize()
        assert sim.check_status() == 0
        x, v, f, tag, typ = sim.host_state()
        vh = v - 0.5 * s.dt * f if k else v
        f_ref, _, _, scale = oracle.forces(s, x, vh, tag, typ, k, with_scale=True)
        if precision == P.FP64:
            _check_fp64(f, f_ref, scale)
        else:
            rel = np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref)
            assert rel <= MIXED_TOL, (s_exp, k, rel)


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_step_with_velocity_prediction(precision):
    """Groot-Warren prediction factor lambda = 0.65 (the forces see
    v~ = v + lambda dt F instead of the half-step velocity): each of 8 steps
    against one oracle step from the GPU's own previous state (positions
    bit-exact, forces within the form's bar), and a 12-step call equal to 12
    one-step calls bit for bit (in the mixed form the predicted velocity is
    then written by the force pass's row epilogue)."""
    s = di.uniform_fluid(2400, (9.0, 10.0, 8.9), 41, lam=0.65)
    sim = _sorted_system(s, precision)
    prev = sim.host_state()
    for k in range(1, 9):
        sim.step(1)
        torch.cuda.synchronize()
        assert sim.check_status() == 0
        cur = sim.host_state()
        xo, vo, fo, _ = oracle.step(s, prev[0], prev[1], prev[2], prev[3], prev[4], k)
        o_prev = np.argsort(prev[3])
        o_cur = np.argsort(cur[3])
        np.testing.assert_array_equal(cur[0][:, o_cur], xo[:, o_prev], err_msg=f"step {k} x")
        vt = prev[1] + s.lam * s.dt * prev[2]
        _, _, _, scale = oracle.forces(s, xo, vt, prev[3], prev[4], k, with_scale=True)
        if precision == P.FP64:
            _check_fp64(cur[2][:, o_cur], fo[:, o_prev], scale[o_prev])
        else:
            rel = np.linalg.norm(cur[2][:, o_cur] - fo[:, o_prev]) / np.linalg.norm(fo)
            assert rel <= MIXED_TOL, (k, rel)
        prev = cur
    a = _sorted_system(s, precision)
    a.step(12)
    b = _sorted_system(s, precision)
    for _ in range(12):
        b.step(1)
    torch.cuda.synchronize()
    for u, w in zip(a.host_state(), b.host_state()):
        np.testing.assert_array_equal(u, w)


def test_step_deterministic_and_resumable():
    s = di.amphiphile(n=6000, seed=2)
    a = _sorted_system(s)
    a.step(20)
    b = _sorted_system(s)
    b.step(20)
    torch.cuda.synchronize()
    for u, w in zip(a.host_state(), b.host_state()):
        np.testing.assert_array_equal(u, w)
    # resume: 10 + 10 steps through a host snapshot equals 20 straight steps
    c = _sorted_system(s)
    c.step(10)
    x, v, f, tag, typ = c.host_state()
    d = P.System(c.params, s.n, P.FP64)
    d.restore(x, v, f, tag, typ, step=10)
    d.step(10)
    torch.cuda.synchronize()
    for u, w in zip(a.host_state(), d.host_state()):
        np.testing.assert_array_equal(u, w)


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_steps_in_one_call_equal_single_step_calls(precision):
    """Inside one dpd_step call the force pass reads the builder's slab (the
    CSR list is written only for the last step); twelve steps in one call
    equal twelve one-step calls bit for bit, lists included."""
    s = di.amphiphile(n=6000, seed=21)
    a = _sorted_system(s, precision)
    a.step(12)
    b = _sorted_system(s, precision)
    for _ in range(12):
        b.step(1)
    torch.cuda.synchronize()
    for u, w in zip(a.host_state(), b.host_state()):
        np.testing.assert_array_equal(u, w)
    for u, w in zip(a.host_nlist(), b.host_nlist()):
        np.testing.assert_array_equal(u, w)


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_step_statistics_match_the_state(precision):
    """Each step's statistics (in the mixed form summed by the force pass's
    row epilogue, which also does the step's half-kicks): a 12-step call
    gives the same rows, bit for bit, as 12 one-step calls, and the last
    row's momentum, sum of v^2 and k_B T equal those of the velocities the
    call leaves (sums taken on the host in a different order)."""
    s = di.amphiphile(n=6000, seed=29)
    a = _sorted_system(s, precision)
    red_a = torch.zeros((12, 8), dtype=torch.float64, device="cuda")
    a.step(12, reductions=red_a)
    b = _sorted_system(s, precision)
    red_b = torch.zeros((12, 8), dtype=torch.float64, device="cuda")
    for k in range(12):
        b.step(1, reductions=red_b[k:k + 1])
    torch.cuda.synchronize()
    assert a.check_status() == 0 and b.check_status() == 0
    np.testing.assert_array_equal(red_a.cpu().numpy(), red_b.cpu().numpy())
    v = a.host_state()[1]
    r = red_a.cpu().numpy()[-1]
    n = v.shape[1]
    p = v.sum(axis=1)
    v2 = float((v * v).sum())
    np.testing.assert_allclose(r[:3], p, rtol=0, atol=1e-11 * np.abs(v).sum())
    np.testing.assert_allclose(r[3], v2, rtol=1e-12)
    kbt = (v2 - float((p * p).sum()) / n) / (3.0 * (n - 1))
    np.testing.assert_allclose(r[6], kbt, rtol=1e-11)


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_step_call_forces_match_oracle_bonded(precision):
    """The path a multi-step dpd_step call runs (list rows read from the
    builder's slab with stencil-coded entries, FP64 pairs inside a chunk
    evaluated once, bond partners carried from reorder to reorder instead of
    looked up by tag), on the bonded amphiphile system: after one 12-step
    call the returned forces equal the oracle's forces at the final state
    (x, v_h = v - dt/2 F, step 12), FP64 within 1e-12 S_i per particle, the
    mixed form within 1e-5 of |F| (global L2 and 99.99th percentile)."""
    s = di.amphiphile(n=6000, seed=23)
    sim = _sorted_system(s, precision)
    red = torch.zeros((12, 8), dtype=torch.float64, device="cuda")
    sim.step(12, reductions=red)
    torch.cuda.synchronize()
    assert sim.check_status() == 0
    x, v, f, tag, typ = sim.host_state()
    vh = v - 0.5 * s.dt * f
    f_ref, pe_ref, npair_ref, scale = oracle.forces(s, x, vh, tag, typ, 12, with_scale=True)
    if precision == P.FP64:
        _check_fp64(f, f_ref, scale)
    else:
        rel = np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref)
        assert rel <= MIXED_TOL, rel
        d = np.linalg.norm(f - f_ref, axis=0)
        rms = np.sqrt(np.mean(np.sum(f_ref**2, axis=0)))
        assert np.percentile(d / rms, 99.99) <= MIXED_TOL
    # the last step's statistics: pair count and potential energy
    r = red.cpu().numpy()[-1]
    assert r[5] == npair_ref.sum() / 2
    np.testing.assert_allclose(r[4], pe_ref.sum(), rtol=1e-12 if precision == P.FP64 else 1e-5)
    # the CSR list the call leaves (its last step's rows) is the oracle's
    off, idx = sim.host_nlist()
    off_ref, idx_ref = oracle.neighbors(x, s.box, s.r_c)
    np.testing.assert_array_equal(off, off_ref)
    np.testing.assert_array_equal(idx, idx_ref)


def test_step_mixed_tracks_fp64():
    s = di.small_fluid(4)
    a = _sorted_system(s, precision=P.MIXED)
    red = torch.zeros((1, 8), dtype=torch.float64, device="cuda")
    prev = a.host_state()
    for k in range(1, 11):
        a.step(1, reductions=red)
        torch.cuda.synchronize()
        cur = a.host_state()
        # the mixed step's forces against the FP64 oracle at the same state;
        # they were evaluated with the half-step velocity v_h = v - dt/2 F
        vh = cur[1] - 0.5 * s.dt * cur[2]
        f_ref, _, _ = oracle.forces(s, cur[0], vh, cur[3], cur[4], k)
        rel = np.linalg.norm(cur[2] - f_ref) / np.linalg.norm(f_ref)
        assert rel <= MIXED_TOL, (k, rel)
        prev = cur


# --------------------------------------------------------------- adjoint --

@pytest.mark.parametrize("name", ["fluid3000", "amphiphile"])
def test_forces_backward_matches_oracle(name):
    s = _systems()[name]
    sim = _sorted_system(s)
    x, v, f, tag, typ = sim.host_state()
    rng = np.random.default_rng(0)
    g = rng.standard_normal(x.shape)
    nt = s.n_types
    gx = torch.empty((3, s.n), dtype=torch.float64, device="cuda")
    gv = torch.empty_like(gx)
    ga = torch.empty(nt * nt, dtype=torch.float64, device="cuda")
    gg = torch.empty_like(ga)
    P.dpd_forces_backward(sim.params, sim.state, sim.cells, sim.nlist, 5,
                          torch.as_tensor(g, device="cuda"), gx, gv, ga, gg, sim.ws)
    torch.cuda.synchronize()
    xb, vb, ab, gb = oracle.forces_vjp(s, x, v, tag, typ, 5, g)
    np.testing.assert_allclose(gx.cpu().numpy(), xb, rtol=1e-9, atol=1e-9 * np.abs(xb).max())
    np.testing.assert_allclose(gv.cpu().numpy(), vb, rtol=1e-9, atol=1e-9 * np.abs(vb).max())
    np.testing.assert_allclose(ga.cpu().numpy().reshape(nt, nt), ab, rtol=1e-10)
    np.testing.assert_allclose(gg.cpu().numpy().reshape(nt, nt), gb, rtol=1e-10)
