"""MI355X-native merged-index approximate vector join (libvj).

The library computes the batched epsilon-range join of a query set against a
data set over one merged proximity graph (the merged index of the paper,
Section 4.3), with hand-written HIP kernels for gfx950 behind the C ABI in
include/vj.h.  ``vj`` is the ctypes binding of that ABI.
"""
from .vj import (Index, Pairs, VJError, join_params, vj_bruteforce_join,  # noqa: F401
                 vj_build_merged_index, vj_index_from_graph, vj_join, vj_last_error)
