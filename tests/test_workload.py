"""The seeded input generators: the torch stream equals the numpy stream,
and members and non-members are distinct."""
import numpy as np
import pytest

from paper_2411_12365_amd import workload as W

torch = pytest.importorskip("torch")


@pytest.mark.parametrize("seed,start,count", [
    (3, 0, 1000), (0, 10 ** 9, 5000), (2 ** 64 - 1, 12345, 3000), (1004, 7, 4096),
])
def test_torch_stream_equals_numpy_stream(seed, start, count):
    got = W.splitmix64_device(seed, start, count, "cpu", chunk=1000).numpy().view(np.uint64)
    assert np.array_equal(got, W.splitmix64(seed, start, count))


def test_members_and_non_members_are_distinct():
    k = W.keys(200_000, 5)
    q = W.non_members(200_000, 100_000, 5)
    assert len(np.unique(k)) == len(k)
    assert not np.isin(q, k).any()
