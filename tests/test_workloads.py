"""The seeded input generators produce what they promise (no GPU, no container arithmetic)."""
import numpy as np
import pytest

from paper_1908_05936_amd.workloads import large_table, pack_int3, plain_table, splitmix64, zipf_ranks, rng_for


def test_splitmix64_published_vector():
    # reference output of splitmix64 seeded with 1234567 (Vigna's reference implementation)
    assert splitmix64(1234567, 0, 3).tolist() == [6457827717110365317, 3203168211198807973,
                                                   9817491932198370423]
    assert splitmix64(1234567, 2, 1).tolist() == [9817491932198370423]


@pytest.mark.parametrize("N,s", [(1000, 1.1), (40, 1.0), (7, 2.5), (1 << 26, 1.1)])
def test_zipf_rank_frequencies(N, s):
    """Rank frequencies against the exact probabilities k^-s / H(N, s): every one of the top ranks
    and the mass of the rest within 5 standard errors; the extreme ranks occur."""
    rng = rng_for(5)
    n = 400000
    r = zipf_ranks(rng, n, N, s)
    assert r.min() >= 1 and r.max() <= N
    top = min(N, 50)
    k = np.arange(1, top + 1, dtype=np.float64)
    if N <= 10**6:
        H = (np.arange(1, N + 1, dtype=np.float64) ** -s).sum()
    else:   # the head summed exactly, the tail by the Euler-Maclaurin integral
        m = 10**6
        H = (np.arange(1, m + 1, dtype=np.float64) ** -s).sum()
        H += ((N + 0.5) ** (1 - s) - (m + 0.5) ** (1 - s)) / (1 - s)
    p = k ** -s / H
    freq = np.bincount(r, minlength=top + 1)[1:top + 1] / n
    assert np.all(np.abs(freq - p) < 5 * np.sqrt(p * (1 - p) / n) + 1e-5)
    rest = 1.0 - p.sum()
    if rest > 0:
        assert abs((r > top).mean() - rest) < 5 * np.sqrt(rest * (1 - rest) / n) + 1e-5
    if N <= 50:
        assert r.max() == N


def test_plain_table_shape():
    w = plain_table(seed=1, log2_keys=10, log2_capacity=11)
    k = w["insert_keys"]
    assert np.unique(k).size == k.size == 1024
    assert np.isin(w["find1"], k).sum() == 512
    assert np.isin(w["erase"], k).all() and np.unique(w["erase"]).size == 256
    assert np.array_equal(np.sort(w["find2"]), np.sort(k))


def test_large_table_shape():
    w = large_table(seed=3, log2_keys=14, log2_queries=15, log2_churn=12)
    k = w["insert_keys"]
    assert np.unique(k).size == k.size
    assert w["capacity"] == round((1 << 14) / 0.8)
    present = np.isin(w["find"], k)
    assert present.sum() == (1 << 15) - round((1 << 15) * 0.2)
    assert not np.isin(w["reinsert_keys"], k).any()
    assert not np.isin(w["find"][~present], w["reinsert_keys"]).any()


def test_pack_int3_fields():
    assert int(pack_int3(1, 0, 0)) == 1
    assert int(pack_int3(0, 1, 0)) == 1 << 21
    assert int(pack_int3(0, 0, 1)) == 1 << 42
    assert int(pack_int3(-1, 0, 0)) == (1 << 21) - 1
    assert int(pack_int3(0, 0, -1)) == ((1 << 21) - 1) << 42


def test_serving_requests_threaded_equal_sequential():
    from paper_1908_05936_amd.workloads import Serving
    a = Serving(seed=3, n_tables=5, entries_log2=(8, 12), req_log2=(2, 9), rank_pool=1 << 12)
    b = Serving(seed=3, n_tables=5, entries_log2=(8, 12), req_log2=(2, 9), rank_pool=1 << 12)
    one = [a.request() for _ in range(40)]
    many = b.requests(40, threads=4)
    kinds = set()
    for x, y in zip(one, many):
        assert x[:3] == y[:3]
        np.testing.assert_array_equal(x[3], y[3])
        assert (x[4] is None) == (y[4] is None)
        if x[4] is not None:
            np.testing.assert_array_equal(x[4], y[4])
            assert int(x[4][0]) >> 32 == x[0]
        u = a.universe[x[1]]
        allowed = set(a.resident(x[1], 0, u).tolist())   # keys come from the table's universe
        assert set(x[3].tolist()) <= allowed
        kinds.add(x[2])
    assert kinds == {"insert", "find", "erase"}
