"""Shared helpers of the GPU parity tests: oracle recompute on an edge list tracked here."""
import numpy as np

from oracle import graph as Gr
from oracle import simrank as O


class EdgeTracker:
    """Current edge list (oracle side), updated alongside the GPU context."""

    def __init__(self, n, src, dst):
        self.n = n
        self.es = set(zip(np.asarray(src).tolist(), np.asarray(dst).tolist()))

    def apply(self, i, j, op):
        if op > 0:
            assert (i, j) not in self.es
            self.es.add((i, j))
            self.n = max(self.n, i + 1, j + 1)
        else:
            self.es.remove((i, j))

    def arrays(self):
        e = sorted(self.es, key=lambda t: (t[1], t[0]))
        return (np.asarray([a for a, _ in e], dtype=np.int64),
                np.asarray([b for _, b in e], dtype=np.int64))

    def Q(self):
        s, d = self.arrays()
        return Gr.transition_matrix(self.n, s, d)

    def exact(self, C):
        return O.fixed_point(self.Q(), C)


def maxabs(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))))
