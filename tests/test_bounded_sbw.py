"""Bounded serial-bandwidth access patterns (section 4.3) from the oracle,
checked by an independent reading of what such a pattern must satisfy:

* every vertex is executed by exactly one load;
* when a load executes a vertex, each of its neighbours is loaded in the
  same part (the on-chip window holds one part at a time);
* the serial bandwidth of each part, E(t) - S(t) maximised over its loads
  (s/e: first and last position of an executed vertex's closed
  neighbourhood inside the part, the load itself for loads that only
  deliver a ghost; S suffix minimum of s, E prefix maximum of e -- the
  section 4.1 definition the oracle's bandwidth() uses), is at most the
  bound.

With a bound at or above AM1's own serial bandwidth, the pattern is the AM1
order in one part (the k = 1 rows of the paper's table of bounded runs).
"""

import numpy as np
import pytest

import oracle
from fvgen.mesh import periodic_mesh, shuffled_periodic_mesh


from pins import pattern_sbw as check_pattern


def distinct(nbr, v):
    return sorted({int(w) for w in nbr[v] if w != v})


def test_checker_reads_a_permutation_like_the_oracle():
    m = shuffled_periodic_mesh(12)
    perm = oracle.am1_order(m.nbr)
    label = np.empty_like(perm)
    label[perm] = np.arange(m.n, dtype=np.int32)
    pat = {"idx": perm, "ex": np.ones(m.n, np.uint8), "part_begin": np.array([0, m.n])}
    assert check_pattern(m.nbr, pat) == oracle.bandwidth(m.nbr, label)["S_BW"]


@pytest.mark.parametrize("N,jitter", [(12, 0.2), (20, 0.0), (32, 0.2)])
def test_bound_at_am1_bandwidth_gives_the_am1_order(N, jitter):
    m = periodic_mesh(N, jitter=jitter)
    perm = oracle.am1_order(m.nbr)
    label = np.empty_like(perm)
    label[perm] = np.arange(m.n, dtype=np.int32)
    sbw = oracle.bandwidth(m.nbr, label)["S_BW"]
    pat = oracle.am1_bounded(m.nbr, sbw)
    assert len(pat["part_begin"]) == 2
    assert np.array_equal(pat["idx"], perm) and np.all(pat["ex"] == 1)
    assert np.all(pat["perfect"] == 1)


@pytest.mark.parametrize("frac", [0.9, 0.6, 0.35, 0.15])
def test_smaller_bounds_hold_with_reloads(frac):
    m = shuffled_periodic_mesh(24)
    perm = oracle.am1_order(m.nbr)
    label = np.empty_like(perm)
    label[perm] = np.arange(m.n, dtype=np.int32)
    sbw = oracle.bandwidth(m.nbr, label)["S_BW"]
    bound = max(4, int(frac * sbw))
    pat = oracle.am1_bounded(m.nbr, bound)
    got = check_pattern(m.nbr, pat)
    assert got <= bound, (got, bound)
    parts = len(pat["part_begin"]) - 1
    k = len(pat["idx"]) / m.n
    assert parts > 1 and k > 1.0
    # a perfect vertex has all its neighbours executed by the end of its part
    done_at = np.empty(m.n, np.int64)
    exec_pos = np.nonzero(pat["ex"])[0]
    done_at[pat["idx"][exec_pos]] = np.searchsorted(pat["part_begin"], exec_pos, side="right")
    for v in np.nonzero(pat["perfect"])[0][:200]:
        assert all(done_at[w] <= done_at[v] for w in distinct(m.nbr, v))


def test_rejects_a_bound_not_above_the_degree():
    m = periodic_mesh(4)
    with pytest.raises(RuntimeError):
        oracle.am1_bounded(m.nbr, 3)
