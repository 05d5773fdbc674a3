"""dpd_forces_noalloc (the force entry point that allocates nothing: its
per-workgroup partials live in the library's static device array) against
dpd_forces with a caller workspace, through the C ABI: forces, per-particle
potential energies and the (PE, pairs) totals bit for bit, in both
precisions, on two calls in a row, the second on a smaller system (so the
second call reads fewer partials than the first left in the array)."""
import numpy as np
import pytest

import dpd_inputs as di

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1311_0402_amd")
from paper_1311_0402_amd import dpd as D  # noqa: E402


def _loaded(s, precision):
    sim = P.System(P.Params.like(s), s.n, precision)
    sim.load(s.x, s.v, s.tag, s.type, step=0)
    torch.cuda.synchronize()
    assert sim.check_status() == 0
    return sim


def _both(sim, step):
    mixed = sim.precision == P.MIXED
    kw = dict(x32=sim.x32 if mixed else None, v32=sim.v32 if mixed else None)
    n = sim.n
    out = []
    for noalloc in (False, True):
        f = torch.full((3, n), np.nan, dtype=torch.float64, device="cuda")
        pe = torch.full((n,), np.nan, dtype=torch.float64, device="cuda")
        stats = torch.full((2,), np.nan, dtype=torch.float64, device="cuda")
        if noalloc:
            D.dpd_forces_noalloc(sim.params, sim.precision, sim.state, sim.cells, sim.nlist, step, f,
                                 pe_out=pe, stats=stats, status=sim.status, **kw)
        else:
            D.dpd_forces(sim.params, sim.precision, sim.state, sim.cells, sim.nlist, step, f, sim.ws,
                         pe_out=pe, stats=stats, status=sim.status, **kw)
        torch.cuda.synchronize()
        out.append((f.cpu().numpy(), pe.cpu().numpy(), stats.cpu().numpy()))
    return out


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_noalloc_forces_equal_workspace_forces(precision):
    big = di.amphiphile(n=60_000, seed=41)          # bonds: the status word is used too
    small = di.small_fluid(42)                       # 3,000 particles: a smaller force grid
    for s, step in ((big, 7), (small, 8)):
        sim = _loaded(s, precision)
        (f0, pe0, st0), (f1, pe1, st1) = _both(sim, step)
        assert np.all(np.isfinite(f0)) and np.all(np.isfinite(st0))
        np.testing.assert_array_equal(f1, f0)
        np.testing.assert_array_equal(pe1, pe0)
        np.testing.assert_array_equal(st1, st0)
        assert st0[1] > 0.5 * s.n                    # pairs inside r_c were counted
        assert sim.check_status() == 0


def test_noalloc_rejects_bad_arguments():
    s = di.small_fluid(43)
    sim = _loaded(s, P.FP64)
    f = torch.empty((3, s.n), dtype=torch.float64, device="cuda")
    with pytest.raises(P.DPDError):
        D.dpd_forces_noalloc(sim.params, 7, sim.state, sim.cells, sim.nlist, 0, f)
