"""Failure paths of the device status word, forced from the host with
inputs every kernel handles without faulting: a non-finite velocity (the
particle's position becomes NaN, it is binned into cell 0 and no distance
test accepts it, so it has no neighbours; the step's totals become NaN), a
bond partner tag with no particle (looked up as "missing", never used as an
index), and a neighbour list too small for a later step of a multi-step
call (the call keeps running with the list discarded; the caller replays
it from the state it entered with)."""
import numpy as np
import pytest

import dpd_inputs as di

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
P = pytest.importorskip("paper_1311_0402_amd")
from paper_1311_0402_amd import _abi  # noqa: E402


def _loaded(s, precision=P.FP64, capacity=None):
    sim = P.System(P.Params.like(s), s.n, precision, capacity=capacity)
    sim.load(s.x, s.v, s.tag, s.type, step=0)
    torch.cuda.synchronize()
    return sim


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_nonfinite_velocity_sets_status_and_raises(precision):
    s = di.small_fluid(6)
    sim = _loaded(s, precision)
    assert sim.check_status() == 0
    x, v, f, tag, typ = sim.host_state()
    v = v.copy()
    v[1, 17] = np.nan
    sim.restore(x, v, f, tag, typ, step=0)
    red = torch.zeros((2, 8), dtype=torch.float64, device="cuda")
    sim.step(2, reductions=red)
    torch.cuda.synchronize()
    st = int(sim.status.item())
    assert st & _abi.STATUS_NONFINITE
    assert not st & _abi.STATUS_NLIST_OVERFLOW
    assert not np.all(np.isfinite(red.cpu().numpy()[:, :5]))
    with pytest.raises(P.DPDError, match="non-finite"):
        sim.check_status()
    # the other particles still have finite forces
    xs, vs, fs, ts, _ = sim.host_state()
    bad = np.nonzero(ts == tag[17])[0]
    others = np.setdiff1d(np.arange(s.n), bad)
    assert np.all(np.isfinite(xs[:, others]))


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_missing_bond_partner_sets_status_and_raises(precision):
    s = di.amphiphile(n=6000, seed=24)
    partner = s.partner.copy()
    head = 4 * 17                                   # a chain's first bead
    partner[head, 1] = s.n + 7                      # a tag no particle has
    s.partner = partner
    sim = _loaded(s, precision)                     # dpd_forces: lookup through idx_of_tag
    assert int(sim.status.item()) & _abi.STATUS_BAD_BOND
    with pytest.raises(P.DPDError, match="bond partner"):
        sim.check_status()
    sim.status.zero_()
    sim.step(3)                                     # dpd_step: partners carried by index
    torch.cuda.synchronize()
    assert int(sim.status.item()) & _abi.STATUS_BAD_BOND
    with pytest.raises(P.DPDError, match="bond partner"):
        sim.check_status()


def _converging_fluid():
    """A 3,000-particle fluid whose velocities point at the box centre: the
    central density (and with it the neighbour count) grows step by step."""
    s = di.small_fluid(7)
    centre = (np.asarray(s.box, dtype=np.float64) / 2.0)[:, None]
    s.v = s.v - 0.8 * (s.x - centre)
    return s


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_overflow_inside_a_call_is_replayed_bitwise(precision):
    s = _converging_fluid()
    ref = _loaded(s, precision)
    n0 = int(ref.nlist.offset[s.n].item())
    red_ref = torch.zeros((10, 8), dtype=torch.float64, device="cuda")
    assert ref.advance(10, reductions=red_ref) == 0
    n10 = int(ref.nlist.offset[s.n].item())
    assert n10 > n0 * 1.02, (n0, n10)               # the list did grow
    tight = _loaded(s, precision, capacity=n0)      # room for the first list only
    assert tight.nlist.capacity == n0
    red = torch.zeros((10, 8), dtype=torch.float64, device="cuda")
    grown = tight.advance(10, reductions=red)
    torch.cuda.synchronize()
    assert grown >= 1
    assert tight.nlist.capacity >= n10
    assert tight.check_status() == 0
    for u, w in zip(ref.host_state(), tight.host_state()):
        np.testing.assert_array_equal(u, w)
    for u, w in zip(ref.host_nlist(), tight.host_nlist()):
        np.testing.assert_array_equal(u, w)
    np.testing.assert_array_equal(red.cpu().numpy(), red_ref.cpu().numpy())
    assert tight.step_count == 10
