"""Host-side checks of libdpd that need no GPU: the library loads, exports
every entry point include/dpd.h declares, validates arguments before
enqueuing anything, and its cell-ranking rule equals the oracle's."""
import ctypes as C
import os
import re
import subprocess
import tempfile

import numpy as np
import pytest

import dpd_inputs as di
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dpd.h")

P = pytest.importorskip("paper_1311_0402_amd")
from paper_1311_0402_amd import _abi  # noqa: E402


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dpd_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    names = _declared()
    assert {"dpd_bin_reorder", "dpd_build_neighbors", "dpd_forces", "dpd_step",
            "dpd_forces_backward"} <= set(names)
    lib = _abi.lib()
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_abi.SIGNATURES)
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    for n in names:
        assert re.search(rf"\bT {n}$", out, flags=re.M), n


def _params(**kw):
    s = di.small_fluid(1)
    p = P.Params.like(s, device="cpu")
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_cell_grid_matches_oracle_rule():
    for box in [(10.0, 10.0, 10.0), (174.716, 174.716, 174.716), (20.0, 40.0, 20.0),
                (80.0, 80.0, 80.0 / 3.0), (3.0000001, 5.0, 7.25)]:
        p = _params(box=box)
        assert P.cell_grid(p) == tuple(oracle.cell_grid(box, 1.0))
    with pytest.raises(P.DPDError):
        P.cell_grid(_params(box=(3.0, 10.0, 10.0)))


@pytest.mark.parametrize("bad", [dict(r_c=0.0), dict(dt=-1.0), dict(s=0.0), dict(n_types=0),
                                 dict(skin=-0.1), dict(box=(10.0, float("nan"), 10.0)),
                                 dict(n_types=2, a=np.array([[25.0, 30.0], [31.0, 25.0]]),
                                      gamma=np.full((2, 2), 4.5), sigma=np.full((2, 2), 3.0))])
def test_invalid_params_rejected(bad):
    p = _params(**bad)
    assert _abi.lib().dpd_workspace_bytes(C.byref(p.c()), 100, 0) == 0
    st = _abi.dpd_state()
    st.n = 0
    code = _abi.lib().dpd_forces(C.byref(p.c()), 0, C.byref(st), None, None, None,
                                 C.byref(_abi.dpd_nlist()), 0, None, None, None, None, None, 0, None)
    assert code == _abi.DPD_EINVAL
    assert _abi.lib().dpd_last_error().decode()


def test_null_and_size_errors_before_launch():
    p = _params().c()
    lib = _abi.lib()
    assert lib.dpd_step(C.byref(p), 0, None, 1, None, None, None, None, None, None, None, None, None,
                        0, None) == _abi.DPD_EINVAL
    st = _abi.dpd_state()
    st.n = 10                    # arrays missing
    assert lib.dpd_bin_reorder(C.byref(p), C.byref(st), C.byref(st), None, None, None, None, 0,
                               None) == _abi.DPD_EINVAL
    assert b"NULL" in lib.dpd_last_error()
    assert lib.dpd_forces(C.byref(p), 7, C.byref(st), None, None, None, None, 0, None, None, None,
                          None, None, 0, None) == _abi.DPD_EINVAL
    # workspace too small -> ECAPACITY (all other arguments are plausible host
    # addresses; nothing is launched because validation fails first)
    n = 10
    buf = [np.zeros(3 * n) for _ in range(3)]
    st.x, st.v, st.f = (b.ctypes.data for b in buf)
    tags = np.zeros(n, dtype=np.uint32); types = np.zeros(n, dtype=np.uint8)
    st.tag, st.type = tags.ctypes.data, types.ctypes.data
    cells = _abi.dpd_cells()
    cs = np.zeros(1000, dtype=np.int32)
    cells.cell_start = cells.cell_xyz = cells.perm = cs.ctypes.data
    nl = _abi.dpd_nlist()
    nl.capacity = 100
    nl.offset = nl.index = cs.ctypes.data
    d_step = np.zeros(1, dtype=np.uint64)
    ws = np.zeros(1024, dtype=np.uint8)
    wsp = (ws.ctypes.data + 255) // 256 * 256
    x32 = np.zeros(3 * n, dtype=np.float32)
    code = lib.dpd_step(C.byref(p), 0, C.byref(st), 1, d_step.ctypes.data, None, C.byref(cells),
                        C.byref(nl), None, None, None, None, wsp, 256, None)
    assert code == _abi.DPD_EINVAL and b"x32" in lib.dpd_last_error()
    code = lib.dpd_step(C.byref(p), 0, C.byref(st), 1, d_step.ctypes.data, None, C.byref(cells),
                        C.byref(nl), x32.ctypes.data, None, None, None, wsp, 256, None)
    assert code == _abi.DPD_ECAPACITY
    assert b"workspace" in lib.dpd_last_error()


def test_process_wide_settings_validate_and_return_the_previous_value():
    lib = _abi.lib()
    assert lib.dpd_set_list_builder(3) == _abi.DPD_EINVAL
    assert lib.dpd_set_list_builder(-1) == _abi.DPD_EINVAL
    assert lib.dpd_set_list_builder(1) == 0          # default: the tile builder
    assert lib.dpd_set_list_builder(2) == 1
    assert lib.dpd_set_list_builder(0) == 2
    assert lib.dpd_set_pair_evaluation(5) == _abi.DPD_EINVAL
    prev = lib.dpd_set_pair_evaluation(0)
    assert prev == 2                                # default: pairs once in the FP64 form
    assert lib.dpd_set_pair_evaluation(prev) == 0


_RANK_PROBE = r"""
#include <cstdio>
#include "dpd_common.h"
int main() {
  int nx, ny, nz;
  while (std::scanf("%d %d %d", &nx, &ny, &nz) == 3) {
    int nmax = nx > ny ? nx : ny; nmax = nmax > nz ? nmax : nz;
    int nb = dpd::bits_for(nmax);
    for (int z = 0; z < nz; ++z) for (int y = 0; y < ny; ++y) for (int x = 0; x < nx; ++x) {
      int r = dpd::morton_rank(x, y, z, nx, ny, nz, nb);
      int ux, uy, uz;
      dpd::morton_unrank(r, nx, ny, nz, nb, &ux, &uy, &uz);
      if (ux != x || uy != y || uz != z) { std::printf("unrank mismatch\n"); return 1; }
      std::printf("%d\n", r);
    }
  }
}
"""


def test_counting_morton_rank_equals_sorted_rank():
    """The kernels' counting rank (host build of the same header) equals the
    oracle's rank by sorting Morton codes, on power-of-two and ragged grids,
    and the kernels' unrank inverts it."""
    grids = [(9, 9, 9), (8, 8, 8), (5, 3, 6), (17, 4, 33), (3, 3, 3), (20, 39, 19)]
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "r.cpp")
        exe = os.path.join(td, "r")
        open(src, "w").write(_RANK_PROBE)
        subprocess.run(["g++", "-O1", "-std=c++17", "-I",
                        os.path.join(ROOT, "paper_1311_0402_amd", "csrc"), src, "-o", exe], check=True)
        inp = "\n".join(" ".join(map(str, g)) for g in grids)
        out = subprocess.run([exe], input=inp, capture_output=True, text=True, check=True).stdout
    vals = np.array(out.split(), dtype=np.int64)
    at = 0
    for g in grids:
        cnt = int(np.prod(g))
        ref = oracle.morton_rank_table(np.array(g, dtype=np.int32))
        np.testing.assert_array_equal(vals[at:at + cnt], ref)
        at += cnt


_NET_PROBE = r"""
#include <cstdint>
#include <cstdio>
#include "dpd_common.h"
// 0-1 principle, bit-sliced: bit b of word w is input vector (w * 64 + b);
// lane q of that vector is bit q of the vector's number
int main() {
  constexpr dpd::SortNet net = dpd::make_sort_net(27);
  const uint64_t total = 1ull << 27;
  unsigned long long bad = 0;
  for (uint64_t w = 0; w < total / 64; ++w) {
    uint64_t v[27];
    for (int q = 0; q < 27; ++q) {
      uint64_t m = 0;
      for (int b = 0; b < 64; ++b) m |= (((w * 64 + b) >> q) & 1ull) << b;
      v[q] = m;
    }
    for (int c = 0; c < net.count; ++c) {
      const uint64_t x = v[net.a[c]], y = v[net.b[c]];
      v[net.a[c]] = x & y;
      v[net.b[c]] = x | y;
    }
    for (int q = 0; q + 1 < 27; ++q) bad |= v[q] & ~v[q + 1];
  }
  std::printf("%d %llu\n", net.count, bad);
  return 0;
}
"""


def test_stencil_sorting_network_sorts_every_input():
    """The 27-key comparison network the lane list builder sorts its stencil
    with (host build of the same header) sorts all 2^27 zero-one inputs, so by
    the zero-one principle it sorts every input."""
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "n.cpp")
        exe = os.path.join(td, "n")
        open(src, "w").write(_NET_PROBE)
        subprocess.run(["g++", "-O2", "-std=c++17", "-I",
                        os.path.join(ROOT, "paper_1311_0402_amd", "csrc"), src, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True, timeout=300).stdout.split()
    assert int(out[0]) == 156
    assert int(out[1]) == 0


def test_batch_create_validates_before_touching_memory():
    """dpd_batch_create rejects bad batches before any copy or launch: sizes,
    offsets, table size and alignment, bonds, fields systems must share."""
    lib = _abi.lib()
    assert lib.dpd_batch_table_bytes(0, 10) == 0
    assert lib.dpd_batch_table_bytes(3, 2) == 0                 # fewer particles than systems
    assert lib.dpd_batch_table_bytes(70000, 10 ** 6) == 0       # beyond the uint16 system map
    need = lib.dpd_batch_table_bytes(3, 3000)
    assert need > 0
    ps = (_abi.dpd_params * 3)(*[_params().c() for _ in range(3)])
    off = np.array([0, 1000, 2000, 3000], dtype=np.int64)
    fake = 1 << 20                   # 256-aligned address that is never dereferenced
    h = C.c_void_p()

    def create(params, offsets, table=fake, nbytes=need):
        return lib.dpd_batch_create(params, 3, offsets.ctypes.data, table, nbytes, None, C.byref(h))

    assert create(ps, np.array([0, 1000, 1000, 3000], dtype=np.int64)) == _abi.DPD_EINVAL
    assert b"empty" in lib.dpd_last_error()
    assert create(ps, np.array([5, 1000, 2000, 3000], dtype=np.int64)) == _abi.DPD_EINVAL
    assert create(ps, off, table=None) == _abi.DPD_EINVAL
    assert create(ps, off, table=fake + 8) == _abi.DPD_EINVAL
    assert create(ps, off, nbytes=need - 1) == _abi.DPD_ECAPACITY
    bad = (_abi.dpd_params * 3)(*[_params().c() for _ in range(3)])
    bad[1].dt = 0.02
    assert create(bad, off) == _abi.DPD_EUNSUPPORTED
    assert b"system 1" in lib.dpd_last_error()
    partner = np.zeros(2000, dtype=np.int32)
    bonded = (_abi.dpd_params * 3)(*[_params().c() for _ in range(3)])
    bonded[2].bond_partner = partner.ctypes.data
    assert create(bonded, off) == _abi.DPD_EUNSUPPORTED
    small = (_abi.dpd_params * 3)(*[_params().c() for _ in range(3)])
    small[0].box[1] = 2.0
    assert create(small, off) == _abi.DPD_EINVAL
    assert b"system 0" in lib.dpd_last_error()
    assert h.value is None
    lib.dpd_batch_destroy(None)


def test_autotune_staged_search_space():
    """The tile builder ignores nlist_waves, so it is one candidate; the
    force grid is searched once, with the chosen builder."""
    from paper_1311_0402_amd import autotune as A
    b = A.builder_candidates()
    assert sum(1 for t in b if t.nlist_kind == 0) == 1
    assert sorted(t.nlist_waves for t in b if t.nlist_kind == 1) == [1, 2, 4]
    assert sorted(t.nlist_waves for t in b if t.nlist_kind == 2) == [1, 2, 4]
    assert all(t.force_grid == 0 for t in b)
    f = A.force_candidates(b[3])
    assert [t.force_grid for t in f] == list(A.FORCE_GRIDS)
    assert all((t.nlist_kind, t.nlist_waves) == (b[3].nlist_kind, b[3].nlist_waves) for t in f)
    assert len(A.default_candidates()) == len(b) * len(A.FORCE_GRIDS)
