"""The seeded input generators: permutations of 1..n are permutations, and
every generator is a function of its seed alone."""
import numpy as np
import pytest

from paper_1804_10062_amd import inputs


@pytest.mark.parametrize("n", [1, 2, 3, 10, 1000, 4097, (1 << 16) + 1])
def test_permutation_is_a_permutation(n):
    p = inputs.permutation_u32(n, seed=5)
    assert p.dtype == np.uint32
    assert np.array_equal(np.sort(p), np.arange(1, n + 1, dtype=np.uint32))


def test_permutation_depends_on_the_seed_only():
    a = inputs.permutation_u32(5000, seed=3)
    assert np.array_equal(a, inputs.permutation_u32(5000, seed=3))
    assert not np.array_equal(a, inputs.permutation_u32(5000, seed=4))
    # not the identity nor a rotation of it
    assert np.count_nonzero(a == np.arange(1, 5001)) < 50


def test_permutation_zero_length():
    assert inputs.permutation_u32(0, seed=1).size == 0
