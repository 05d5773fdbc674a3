"""Batched replicas on the GPU: every system of a batch equals its own
single-system run bit for bit (state, forces, neighbour rows), whatever the
launch shapes and whether a step runs eagerly or as a captured HIP graph;
per-system statistics equal the single-system ones up to summation order;
one system checked directly against the oracle."""
import numpy as np
import pytest

import dpd_inputs as di
import oracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1311_0402_amd")


def _spec(n_sys=7, seed=41):
    return di.batched_spec(n_sys=n_sys, seed=seed, n_min=1000, n_max=9000)


def _systems(spec):
    return di.batched_systems(spec, seed=3)


def _concat(systems):
    x = np.concatenate([s.x for s in systems], axis=1)
    v = np.concatenate([s.v for s in systems], axis=1)
    tag = np.concatenate([s.tag for s in systems])
    typ = np.concatenate([s.type for s in systems])
    return x, v, tag, typ


def _batch(systems, precision, **kw):
    b = P.Batch([P.Params.like(s) for s in systems], [s.n for s in systems], precision=precision, **kw)
    b.load(*_concat(systems))
    return b


def _single(s, precision):
    sim = P.System(P.Params.like(s), s.n, precision)
    sim.load(s.x, s.v, s.tag, s.type)
    return sim


def _local_rows(off, idx, lo, hi):
    """CSR rows lo..hi-1 with entries shifted to system-local indices."""
    o = off[lo:hi + 1] - off[lo]
    return o, idx[off[lo]:off[hi]] - lo


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_batch_setup_equals_single_systems(precision):
    systems = _systems(_spec())
    b = _batch(systems, precision)
    torch.cuda.synchronize()
    assert b.check_status() == 0
    bx, bv, bf = (t.cpu().numpy() for t in (b.state.x, b.state.v, b.state.f))
    btag = b.state.tag.cpu().numpy().view(np.uint32)
    boff = b.nlist.offset.cpu().numpy().astype(np.int64)
    bidx = b.nlist.index.cpu().numpy().astype(np.int64)
    bperm = b.cells.perm.cpu().numpy()
    bcs = b.cells.cell_start.cpu().numpy()
    c_lo = 0
    for k, s in enumerate(systems):
        sim = _single(s, precision)
        x, v, f, tag, _ = sim.host_state()
        off, idx = sim.host_nlist()
        sl = b.system_slice(k)
        lo, hi = sl.start, sl.stop
        np.testing.assert_array_equal(bx[:, sl], x)
        np.testing.assert_array_equal(bv[:, sl], v)
        np.testing.assert_array_equal(btag[sl], tag)
        np.testing.assert_array_equal(bperm[sl] - lo, sim.cells.perm.cpu().numpy())
        cs = sim.cells.cell_start.cpu().numpy()
        np.testing.assert_array_equal(bcs[c_lo:c_lo + cs.size] - lo, cs)
        c_lo += cs.size - 1
        o, i = _local_rows(boff, bidx, lo, hi)
        np.testing.assert_array_equal(o, off)
        np.testing.assert_array_equal(i, idx)
        np.testing.assert_array_equal(bf[:, sl], f, err_msg=f"system {k}")


def test_batch_forces_match_oracle():
    """One system of the batch against the oracle's FP64 forces."""
    systems = _systems(_spec())
    b = _batch(systems, P.FP64)
    k = 3
    s = systems[k]
    sl = b.system_slice(k)
    x = b.state.x[:, sl].cpu().numpy()
    v = b.state.v[:, sl].cpu().numpy()
    tag = b.state.tag[sl].cpu().numpy().view(np.uint32)
    f = b.state.f[:, sl].cpu().numpy()
    ref, _, _, scale = oracle.forces(s, x, v, tag, s.type[tag], 0, mode="cells", with_scale=True)
    assert np.all(np.abs(f - ref) <= 1e-12 * scale)


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_batch_steps_equal_single_systems(precision):
    systems = _systems(_spec())
    K = 6
    b = _batch(systems, precision)
    red = torch.zeros((K, b.n_sys, 8), dtype=torch.float64, device="cuda")
    b.step(K, reductions=red, use_graph=True)
    torch.cuda.synchronize()
    assert b.check_status() == 0
    assert int(b.d_step.item()) == K
    red = red.cpu().numpy()
    bx, bv, bf = (t.cpu().numpy() for t in (b.state.x, b.state.v, b.state.f))
    # the list the call leaves (written once, after the last step)
    boff = b.nlist.offset.cpu().numpy().astype(np.int64)
    bidx = b.nlist.index.cpu().numpy().astype(np.int64)
    for k, s in enumerate(systems):
        sim = _single(s, precision)
        r1 = torch.zeros((K, 8), dtype=torch.float64, device="cuda")
        sim.step(K, reductions=r1)
        x, v, f, _, _ = sim.host_state()
        sl = b.system_slice(k)
        np.testing.assert_array_equal(bx[:, sl], x, err_msg=f"system {k}")
        np.testing.assert_array_equal(bv[:, sl], v, err_msg=f"system {k}")
        np.testing.assert_array_equal(bf[:, sl], f, err_msg=f"system {k}")
        off, idx = sim.host_nlist()
        o, i = _local_rows(boff, bidx, sl.start, sl.stop)
        np.testing.assert_array_equal(o, off, err_msg=f"system {k} offsets")
        np.testing.assert_array_equal(i, idx, err_msg=f"system {k} rows")
        r1 = r1.cpu().numpy()
        # momentum sums cancel: compare them on the scale of sum |v|
        vscale = np.abs(v).sum()
        np.testing.assert_allclose(red[:, k, :3], r1[:, :3], rtol=0, atol=1e-12 * vscale)
        np.testing.assert_allclose(red[:, k, [3, 5, 6]], r1[:, [3, 5, 6]], rtol=1e-12)
        # potential energy: FP64 pair terms sum to 1e-12 either way; in the
        # mixed form each pair's share is an FP32 value and the batch adds
        # FP32 row sums where the single run adds the pair values in FP64
        np.testing.assert_allclose(red[:, k, 4], r1[:, 4], rtol=1e-12 if precision == P.FP64 else 2e-6)


def test_graph_replay_equals_eager_and_is_resumable():
    systems = _systems(_spec(n_sys=5, seed=43))
    runs = []
    for use_graph in (False, True):
        b = _batch(systems, P.MIXED)
        red = torch.zeros((3, b.n_sys, 8), dtype=torch.float64, device="cuda")
        b.step(3, reductions=red, use_graph=use_graph)
        # eager work between graph replays, then more replays of the same graph
        _ = (b.state.v * 2.0).sum().item()
        red2 = torch.zeros((4, b.n_sys, 8), dtype=torch.float64, device="cuda")
        b.step(4, reductions=red2, use_graph=use_graph)
        torch.cuda.synchronize()
        nnz = int(b.nlist.offset[b.n].item())
        runs.append([t.cpu().numpy() for t in (b.state.x, b.state.v, b.state.f, red, red2, b.nlist.offset,
                                                 b.nlist.index[:nnz])])
        assert int(b.d_step.item()) == 7
        b.close()
    for u, w in zip(*runs):
        np.testing.assert_array_equal(u, w)


def test_tiles_do_not_change_results():
    """Launch shapes and all three list builders give bitwise the same lists
    and trajectories."""
    systems = _systems(_spec(n_sys=5, seed=44))
    ref = None
    for tiles in [P.Tiles(), P.Tiles(force_grid=64, nlist_waves=1), P.Tiles(force_grid=4096, nlist_waves=2),
                  P.Tiles(force_grid=700, nlist_waves=4, nlist_kind=1), P.Tiles(nlist_waves=1, nlist_kind=1),
                  P.Tiles(nlist_waves=2, nlist_kind=2)]:
        b = _batch(systems, P.MIXED)
        b.set_tiles(tiles)
        b.rebuild()
        torch.cuda.synchronize()
        nnz = int(b.nlist.offset[b.n].item())
        lists = [b.nlist.offset.cpu().numpy(), b.nlist.index[:nnz].cpu().numpy()]
        b.step(3, use_graph=True)
        torch.cuda.synchronize()
        out = lists + [t.cpu().numpy() for t in (b.state.x, b.state.v, b.state.f)]
        if ref is None:
            ref = out
        else:
            for u, w in zip(ref, out):
                np.testing.assert_array_equal(u, w, err_msg=str(tiles))
        b.close()


def test_batch_argument_errors():
    systems = _systems(_spec(n_sys=3, seed=45))
    params = [P.Params.like(s) for s in systems]
    params[1].dt = 0.005
    with pytest.raises(P.DPDError, match="differs"):
        P.Batch(params, [s.n for s in systems])
    params = [P.Params.like(s) for s in systems]
    params[2].box = (2.0, 10.0, 10.0)
    with pytest.raises(P.DPDError, match="system 2"):
        P.Batch(params, [s.n for s in systems])
    b = _batch(systems, P.MIXED)
    with pytest.raises(P.DPDError):
        b.set_tiles(P.Tiles(force_grid=10))
    with pytest.raises(P.DPDError):
        b.set_tiles(P.Tiles(nlist_waves=3))
    with pytest.raises(P.DPDError):
        b.set_tiles(P.Tiles(nlist_kind=3))
    assert b.get_tiles() == P.Tiles(0, 4, 0)


def test_autotune_restores_state_and_caches(tmp_path, monkeypatch):
    from paper_1311_0402_amd import autotune
    monkeypatch.setenv("DPD_AUTOTUNE_CACHE", str(tmp_path / "autotune.json"))
    systems = _systems(_spec(n_sys=4, seed=46))
    cands = [P.Tiles(0, 4), P.Tiles(512, 1), P.Tiles(2048, 2, 1)]
    b = _batch(systems, P.MIXED)
    best, timings = autotune.tune(b, candidates=cands, steps=2)
    assert best in cands and len(timings) == len(cands)
    assert b.get_tiles() == P.Tiles(best.force_grid, best.nlist_waves or 4, best.nlist_kind)
    assert int(b.d_step.item()) == 0
    ref = _batch(systems, P.MIXED)
    b.step(3)
    ref.step(3)
    torch.cuda.synchronize()
    for u, w in zip((b.state.x, b.state.v, b.state.f), (ref.state.x, ref.state.v, ref.state.f)):
        assert torch.equal(u, w)
    again, _ = autotune.tune(ref, candidates=[P.Tiles(4096, 1)])
    assert again == best                     # served from the cache
    assert (tmp_path / "autotune.json").exists()
