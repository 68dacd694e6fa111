"""The paper's multithreaded CPU scan (the context leg of the benchmark)
against the oracle: bit-exact for any thread count and partition size,
including partitions that do not divide the array, more threads than
partitions, and in place."""
import numpy as np
import pytest

import oracle
import workloads
import cpu_context


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
@pytest.mark.parametrize("partition", [1, 7, 1000, 1 << 16])
def test_matches_oracle(threads, partition):
    a = workloads.full_u32(200_003, seed=5000 + threads)
    assert np.array_equal(cpu_context.two_pass_scan_u32(a, threads, partition), oracle.scan_int(a))


def test_in_place_and_small():
    for n in (1, 2, 5, 64):
        a = workloads.full_u32(n, seed=5100 + n)
        want = oracle.scan_int(a)
        b = a.copy()
        cpu_context.two_pass_scan_u32(b, 4, 3, out=b)
        assert np.array_equal(b, want), n
