"""MI355X-native per-vertex directed 3-, 4- and 5-motif counting (the VDMC method).

The work runs in the HIP library ``libvdmc.so`` behind the C ABI of ``include/vdmc.h``;
this package is its Python binding (``vdmc.py``) and build script (``build.py``).
"""
from .vdmc import (  # noqa: F401
    Graph,
    Server,
    VdmcError,
    class_codes,
    class_table,
    count,
    count34,
    count_range,
    count_batch,
    count_batch_noalloc,
    count_supported,
    init,
    count_edges,
    count_undirected,
    edge_list,
    kernel_times,
    load,
    num_classes,
    num_classes_undirected,
    profile_counters,
    shape_counts,
    shape_counts5,
    SHAPES5,
    tune,
    tuned_choice,
    set_hub_threshold,
    undirected_classes,
)
