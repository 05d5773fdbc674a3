"""Parity at the benchmark's full size: the 16,000,000-particle amphiphile
system (chains, three types), in the launch configuration bench.py times.

The whole reorder permutation and cell table are compared with the oracle
bit for bit; neighbour rows and forces are compared on a seeded sample of
rows the oracle computes one by one (brute-force rows over all 16M
particles), after one real time step so positions have moved and been
reordered."""
import numpy as np
import pytest

import dpd_inputs as di
import oracle

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.timeout(600)]
P = pytest.importorskip("paper_1311_0402_amd")

N_FULL = 16_000_000
N_SAMPLE = 1000


@pytest.fixture(scope="module")
def full():
    return di.amphiphile(n=N_FULL, seed=3)


def _sample(n, seed=12):
    return np.sort(np.random.default_rng(seed).choice(n, size=N_SAMPLE, replace=False)).astype(np.int32)


def _loaded(s, precision):
    sim = P.System(P.Params.like(s), s.n, precision)
    sim.load(s.x, s.v, s.tag, s.type, step=0)
    torch.cuda.synchronize()
    sim.check_status()
    return sim


def test_fullsize_reorder_is_the_oracle_permutation(full):
    s = full
    sim = _loaded(s, P.FP64)
    perm_ref, cs_ref = oracle.reorder(s.x, s.tag, s.box, 1.0)
    np.testing.assert_array_equal(sim.cells.perm.cpu().numpy(), perm_ref)
    np.testing.assert_array_equal(sim.cells.cell_start.cpu().numpy(), cs_ref)
    del sim
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision", [P.FP64, P.MIXED])
def test_fullsize_rows_and_forces_after_a_step(full, precision):
    s = full
    sim = _loaded(s, precision)
    sim.step(1)
    # re-bin the stepped (already sorted) state so the FP32 copies carry its
    # current velocities, then rebuild the list and evaluate at the step's
    # counter, as the oracle does from the same arrays
    st = sim.state
    sim.reorder_from(P.State(st.x.clone(), st.v.clone(), st.f.clone(), st.tag.clone(), st.type.clone()))
    sim.rebuild()
    sim.compute_forces(1)
    torch.cuda.synchronize()
    sim.check_status()
    x, v, f, tag, typ = sim.host_state()
    q = _sample(s.n)
    # neighbour rows of the sample, bit for bit
    off, idx = sim.host_nlist()
    off_ref, idx_ref = oracle.neighbors(x, s.box, 1.0, query=q)
    for k, i in enumerate(q):
        np.testing.assert_array_equal(idx[off[i]:off[i + 1]], idx_ref[off_ref[k]:off_ref[k + 1]],
                                      err_msg=f"row {i}")
    # forces of the sample (bonds included) at the step's counter
    f_ref, _, _, scale = oracle.forces(s, x, v, tag, typ, 1, query=q, with_scale=True)
    fq = f[:, q]
    if precision == P.FP64:
        d = np.linalg.norm(fq - f_ref, axis=0)
        assert np.all(d <= 1e-12 * scale), float(np.max(d / scale))
    else:
        rel = np.linalg.norm(fq - f_ref) / np.linalg.norm(f_ref)
        assert rel <= 1e-5, rel
    del sim
    torch.cuda.empty_cache()
