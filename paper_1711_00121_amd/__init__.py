"""Incremental all-pairs SimRank on MI355X (gfx950): Python binding of libsimrank.

The library (csrc/, built in-tree into libsimrank.so) implements Yu, Lin, Zhang, McCann,
"Dynamical SimRank Search on Time-Varying Networks": rank-one link updates solved by
K sparse matrix-vector products, affected-area pruning, node insertions, similar-sink
batches, a column-by-column mode, and an edge-weight adjoint.
"""
from .simrank import (Context, SimRankPairs, default_config, device_bytes, mfma_layout_probe,
                      partition, simrank_pairs)

__all__ = ["Context", "SimRankPairs", "default_config", "device_bytes", "mfma_layout_probe",
           "partition", "simrank_pairs"]
