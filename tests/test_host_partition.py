"""The library's graph partitioner (host code behind sr_partition, no GPU work) against the
oracle's independent implementation of the same rule: labels equal on every node."""
import numpy as np
import pytest

import workloads as W
from oracle import partition as Pt


@pytest.mark.parametrize("n,m,parts,seed", [(6, 0, 2, 1), (203, 900, 8, 2), (1000, 6000, 5, 3),
                                            (777, 2000, 1, 4), (300, 2500, 300, 5)])
def test_library_partition_equals_oracle(n, m, parts, seed):
    from paper_1711_00121_amd import partition
    if m:
        s, d, _ = W.communities(n, m, min(parts, 8), 0.05, seed=seed)
    else:
        s = d = np.zeros(0, dtype=np.int32)
    got = partition(n, s, d, parts)
    want = Pt.bfs_partition(n, s, d, parts)
    assert np.array_equal(got, want)


def test_library_partition_rejects_bad_arguments():
    from paper_1711_00121_amd import partition
    from paper_1711_00121_amd._lib import SR_EINVAL, SR_ERANGE, SimRankError
    with pytest.raises(SimRankError) as e:
        partition(10, [0], [1], 0)
    assert e.value.status == SR_EINVAL
    with pytest.raises(SimRankError) as e:
        partition(10, [0], [10], 2)
    assert e.value.status == SR_ERANGE
