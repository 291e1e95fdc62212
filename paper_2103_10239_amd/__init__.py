"""MI355X (gfx950) non-metric neighbour lists and Vicsek alignment.

Implements the data-parallel hot path of one time step of the fundamental
simulation loop in D. M. Sussman, "Non-metric interaction rules in models of
active matter" (arXiv:2103.10239): cell binning, k-nearest (topological) and
cutoff (metric) neighbour lists, and the alignment / move of Eq. (2) and
Eq. (1), as hand-written HIP kernels behind the C ABI of include/nm.h.
"""
from . import nm, workloads  # noqa: F401
from .nm import (NM_E_CAPACITY, NM_E_DEVICE, NM_E_INVAL, NM_E_NOMEM, NM_E_RANGE, NM_MAX_K,  # noqa: F401
                 NM_BLOCK_SUBSTRIPS, NM_MOVE_NEW_HEADING, NM_NOISE_SCALAR, NM_OK, Batch, Grid, NMError, Params, Server, System,
                 Workspace, align_step, bin_step, build_cells, check, knn, knn_align, knn_fov, knn_layout, make_params,
                 metric_list,
                 polar_order, server_job_bytes, step, suggest_cell_w, tune_grid, voronoi, voronoi_check,
                 voronoi_forces, voronoi_update)
