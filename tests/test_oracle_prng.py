"""Pins for the oracle's random draws: Philox4x64-10, the SplitMix64 mixer,
the weighted column sampler and the keyed permutation behind the SCD subsets.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O

MASK = (1 << 64) - 1


@pytest.mark.parametrize("key,ctr", [((0, 0), (0, 0, 0, 0)), ((5, 7), (11, 3, 2, 1)),
                                     ((MASK, 1 << 63), (MASK, MASK, 17, 1 << 40))])
def test_philox_matches_numpy(key, ctr):
    # numpy's Philox bit generator is Philox4x64-10 and increments its counter
    # before producing a block, so start it one below the counter we want.
    c = list(ctr)
    for i in range(4):  # subtract one with borrow (wraps to all-ones)
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = MASK
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(c, dtype=np.uint64))
    ref = bg.random_raw(4)
    assert list(O.philox(ctr, key)) == list(ref)


def test_philox_known_answer_zero():
    # Random123 known-answer vector for philox4x64-10, zero counter and key.
    assert [int(v) for v in O.philox((0, 0, 0, 0), (0, 0))] == [
        0x16554D9ECA36314C, 0xDB20FE9D672D0FDC, 0xD7E772CEE186176B, 0x7E68B68AEC7BA23B]


def test_mix64_splitmix_reference_output():
    # SplitMix64 seeded with 0 returns mix(0x9E3779B97F4A7C15) first.
    assert O.mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF


def test_u01_and_uniform_index_edges():
    assert O.u01(0) == 0.0
    assert O.u01(MASK) == 1.0 - 2.0 ** -53
    for n in (1, 2, 7, 1000, 4096):
        assert O.uniform_index(0, n) == 0
        assert O.uniform_index(MASK, n) == n - 1
        assert O.uniform_index(1 << 63, n) == n // 2


def test_weighted_index_boundaries():
    w = np.array([1.0, 0.0, 2.0, 3.0, 0.0])
    prefix = np.cumsum(w)          # 1, 1, 3, 6, 6
    assert O.weighted_index(prefix, 0.0) == 0
    assert O.weighted_index(prefix, 1 / 6 - 1e-12) == 0
    assert O.weighted_index(prefix, 1 / 6) == 2     # zero-weight column 1 never drawn
    assert O.weighted_index(prefix, 0.5 - 1e-12) == 2
    assert O.weighted_index(prefix, 0.5) == 3
    assert O.weighted_index(prefix, 1.0 - 2.0 ** -53) == 3
    assert O.weighted_index(prefix, 1.0) == 3       # rounding fallback: last positive weight


def test_weighted_draws_follow_column_norms():
    rng = np.random.default_rng(0)
    w = rng.random(20) + 0.05
    j1, j2 = O.rk_indices(seed=9, outer=0, t0=0, count=200000, weights=w)
    expected = w / w.sum() * len(j1)
    for js in (j1, j2):
        counts = np.bincount(js, minlength=len(w))
        assert stats.chisquare(counts, expected).pvalue > 1e-4
    # j1 and j2 of one step are independent draws
    table = np.zeros((20, 20))
    np.add.at(table, (j1, j2), 1)
    assert stats.chi2_contingency(table)[1] > 1e-4


@pytest.mark.parametrize("n", [1, 2, 3, 5, 16, 17, 100, 1000, 1025])
def test_scd_keys_are_distinct_and_carry_the_index(n):
    b = max(1, (n - 1).bit_length())
    for K in (0, 1, 0xDEADBEEF, MASK):
        keys = [O.scd_key(K, n, s) for s in range(n)]
        assert len(set(keys)) == n
        assert [k & ((1 << b) - 1) for k in keys] == list(range(n))
        # the random part is the SplitMix64 stream seeded with K
        s = n // 2
        assert keys[s] >> b == O.mix64((K + (s + 1) * 0x9E3779B97F4A7C15) & MASK) >> b


@pytest.mark.parametrize("n,alpha", [(6, 2), (8, 3), (9, 5)])
def test_scd_subsets_are_uniform(n, alpha):
    # every alpha-subset of [n] equally likely: a multinomial test over all of them
    import itertools
    idx = {c: i for i, c in enumerate(itertools.combinations(range(n), alpha))}
    counts = np.zeros(len(idx))
    trials = 200 * len(idx)
    for t in range(trials):
        a, mem = O.scd_subset(seed=4, outer=0, t=t, n=n, alpha_opt=alpha)
        assert a == alpha and mem.sum() == alpha
        counts[idx[tuple(np.nonzero(mem)[0])]] += 1
    assert stats.chisquare(counts).pvalue > 1e-4


def test_scd_alpha_is_uniform():
    n, trials = 12, 5000
    sizes = []
    for t in range(trials):
        alpha, mem = O.scd_subset(seed=4, outer=1, t=t, n=n, alpha_opt=0)
        assert mem.sum() == alpha and 1 <= alpha <= n
        sizes.append(alpha)
    counts = np.bincount(sizes, minlength=n + 1)[1:]
    assert stats.chisquare(counts, np.full(n, len(sizes) / n)).pvalue > 1e-4


def test_scd_subset_full_alpha_is_everything():
    for t in range(20):
        alpha, mem = O.scd_subset(seed=1, outer=2, t=t, n=37, alpha_opt=37)
        assert alpha == 37 and mem.all()
