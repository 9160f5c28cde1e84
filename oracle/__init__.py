"""Oracle: a plain, slow, obviously correct FP64 CPU implementation of incremental
all-pairs SimRank (Yu, Lin, Zhang, McCann, "Dynamical SimRank Search on Time-Varying
Networks").

This package is TEST INFRASTRUCTURE. Only the test suite, the package smoke check and the
benchmark's CPU-baseline leg may import or run it. The GPU library never imports it, shares
no code with it, and must not fall back to it.

What is here, by module:

* ``graph``        transition matrix Q of a digraph (section 3.1, Li et al.'s model).
* ``simrank``      SimRank S as the unique fixed point of eq (03a): Kronecker solve for tiny
                   graphs, the fixed-point iteration, the series of eq (17) per column, and
                   the PartialSim procedure of section 7.
* ``incremental``  dense evaluations of the paper's update formulas, in the paper's order
                   and notation: Theorems 1, 2, 3, 9 (unit link updates), Algorithm 1
                   (Inc-uSR), Theorem 4 (affected areas), Theorems 5-8 and Algorithms 3-5
                   (node insertions C1-C3), Table 2 and Algorithm 6 (batches), Algorithm 7
                   (column-by-column updates).
* ``tree``         all-pairs SimRank seeded from a breadth-first spanning forest (Example
                   1.2): the forest, its S by the example's closed form, and the other edges
                   applied as one Inc-bSR batch.
* ``partition``    all-pairs SimRank over a partitioned graph (Example 1.1): a breadth-first
                   partitioner, S of the blocks computed block by block, and the cross-block
                   edges applied as one Inc-bSR batch.
* ``serving``      top-k single-source selection on a column of S and precision@k.
* ``adjoint``      gradient of a pairwise squared loss on S with respect to edge weights,
                   by the transposed Sylvester iteration, and its finite-difference check.
                   The paper has no gradient; this follows from eq (03a) by the chain rule.

Every function states the passage it follows. Floating point is float64 throughout.
"""
