"""MI355X (gfx950) DPD hot path: HIP kernels behind a C ABI (include/dpd.h).

The package holds the HIP sources (``csrc/``), the build step (``build``),
the ctypes declarations (``_abi``) and the torch binding (``dpd``).  Every
numerical step runs in libdpd.so; importing the binding raises if the
library was not built.
"""
from .dpd import (FP64, MIXED, Batch, Cells, NList, Params, State, System, Tiles, alloc_workspace,
                  border_workspace, cell_grid, default_capacity, dpd_bin_reorder, dpd_border_lists,
                  dpd_border_pack, dpd_border_unpack, dpd_build_neighbors, dpd_forces, dpd_forces_backward,
                  dpd_step, dpd_step_backward, ghost_records, set_list_builder, set_pair_evaluation,
                  workspace_bytes)
from ._abi import DPDError

__all__ = ["FP64", "MIXED", "Batch", "Cells", "NList", "Params", "State", "System", "Tiles", "alloc_workspace",
           "border_workspace", "dpd_border_lists", "dpd_border_pack", "dpd_border_unpack", "ghost_records",
           "cell_grid", "default_capacity", "dpd_bin_reorder", "dpd_build_neighbors", "dpd_forces",
           "dpd_forces_backward", "dpd_step", "dpd_step_backward", "set_list_builder", "set_pair_evaluation",
           "workspace_bytes", "DPDError"]
