"""MI355X (gfx950) population graph-colouring hot path.

The search runs in ``libdlmcol.so`` (hand-written HIP kernels behind the C
ABI declared in ``include/dlmcol.h``); this package only marshals
arguments.  Import fails loudly when the library has not been built.
"""
from ._abi import (  # noqa: F401
    DlmError,
    Graph,
    InvNet,
    MultiBatch,
    NSTATS,
    Scorer,
    abi_version,
    evaluate,
    gather_distances,
    gemm_bf16,
    wvcp_targets,
    gather_pool,
    gather_rows,
    nearest,
    partition_distance,
    spacing_update,
    pop_update,
    probe_lds_bandwidth,
    random_pairs,
    reduce_colours,
    standardize,
    gpx_batch,
    select,
    select_groups,
    init_population,
    invnet_names,
    lib,
    tabu_batch,
    tabu_batch_static,
    tabu_workspace_bytes,
    wvcp_batch,
)
