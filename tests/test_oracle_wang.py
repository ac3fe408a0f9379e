"""Oracle pins for the permutation pairing of Wang et al. (Sec. III D), CPU only.

* The random permutations are the index order of the 64-bit Philox keys
  (keys rebuilt from the Philox block, which is pinned against an external
  implementation elsewhere), and over many temperatures every permutation of
  a small population turns up about equally often.
* The repair is checked by brute force on small populations: its output is
  a permutation without incestuous pairs; it leaves an already valid
  permutation alone; it reports failure exactly when no valid permutation
  exists (a family above R/2, found by enumerating all permutations); the
  "smallest mismatched index first" statement equals a single pass with the
  identity search pattern (the paper recovers the original algorithm by
  fixing sigma = id); the original algorithm is not uniform over the valid
  permutations while the random search pattern makes it so (both stated in
  the paper, checked exhaustively over every pi and sigma).
* The measurement sums, over the repaired pairs (k, pi_k), recomputed with
  numpy from the population's spins equal the oracle's records, and a
  population with a family above R_i/2 gets no pairs.
"""
import collections
import itertools
import math

import numpy as np
import pytest

import oracle
import workloads as W


def keys_of(seed, i, pop, R, which):
    key = [seed & 0xFFFFFFFF, seed >> 32]
    out = []
    for k in range(R):
        o = oracle.philox4x32_10([k, 0, i, (6 << 28) | (pop << 24)], key)
        lo, hi = (o[0], o[1]) if which == 0 else (o[2], o[3])
        out.append(int(lo) | (int(hi) << 32))
    return out


@pytest.mark.parametrize("which", [0, 1])
def test_permutation_is_key_order(which):
    seed, i, pop, R = 0x1234_5678_9ABC, 7, 1, 300
    keys = keys_of(seed, i, pop, R, which)
    want = sorted(range(R), key=lambda k: (keys[k], k))
    got = oracle.random_permutation(seed, i, pop, R, which)
    assert list(got) == want


def test_permutations_of_four_are_equally_likely():
    counts = collections.Counter(tuple(oracle.random_permutation(99, i, 0, 4)) for i in range(4800))
    assert len(counts) == 24
    # chi-square with 23 degrees of freedom; 60 is far in the upper tail
    chi2 = sum((c - 200) ** 2 / 200 for c in counts.values())
    assert chi2 < 60, chi2


def families(sizes):
    return np.repeat(np.arange(len(sizes)), sizes).astype(np.int32)


def valid(fam, p):
    return all(fam[p[k]] != fam[k] for k in range(len(fam)))


@pytest.mark.parametrize("sizes", [[1, 1], [2, 1, 1], [2, 2, 1], [3, 1, 1, 1], [2, 2, 2], [3, 3],
                                   [1, 1, 1, 1, 1], [3, 2, 1], [4, 1, 1], [2, 1], [1]])
def test_repair_against_brute_force(sizes):
    fam = families(sizes)
    R = len(fam)
    perms = [np.array(p, np.int32) for p in itertools.permutations(range(R))]
    any_valid = any(valid(fam, p) for p in perms)
    assert any_valid == (2 * max(sizes) <= R)
    for p in perms:
        st, q = oracle.wang_repair(fam, p)
        if not any_valid:
            assert st == 1 and np.array_equal(q, p)
            continue
        assert st == 0
        assert sorted(q) == list(range(R))          # a permutation
        assert valid(fam, q)                         # no incestuous pair
        if valid(fam, p):
            assert np.array_equal(q, p)              # nothing to repair
        # the original algorithm is the random-pattern one with sigma = id
        st2, q2 = oracle.wang_repair(fam, p, np.arange(R, dtype=np.int32))
        assert st2 == 0 and np.array_equal(q, q2)


def output_distribution(fam, with_sigma):
    R = len(fam)
    perms = [np.array(p, np.int32) for p in itertools.permutations(range(R))]
    c = collections.Counter()
    for p in perms:
        for s in (perms if with_sigma else [None]):
            st, q = oracle.wang_repair(fam, p, s)
            assert st == 0
            c[tuple(q)] += 1
    return c


@pytest.mark.parametrize("sizes", [[2, 2, 1], [2, 1, 1], [3, 1, 1, 1]])
def test_random_search_pattern_restores_uniformity(sizes):
    fam = families(sizes)
    R = len(fam)
    n_valid = sum(valid(fam, p) for p in itertools.permutations(range(R)))
    rdm = output_distribution(fam, True)
    assert len(rdm) == n_valid
    assert len(set(rdm.values())) == 1                 # every valid pairing equally often
    assert sum(rdm.values()) == math.factorial(R) ** 2


def test_original_algorithm_is_not_uniform():
    fam = families([2, 2, 1])
    ident = output_distribution(fam, False)
    n_valid = sum(valid(fam, p) for p in itertools.permutations(range(5)))
    assert len(ident) == n_valid                      # every valid pairing is reachable
    assert max(ident.values()) > 4 * min(ident.values())


def test_pairs_on_a_population_match_numpy():
    d = W.run_desc(8, W.EA_PMJ, seed=W.RUN_SEED_BASE + 0x3300, disorder_seed=W.DISORDER_SEED_BASE + 3,
                   R=300, theta=1, K=14, beta_f=2.5, resampling=W.NEAREST_INT, overlap=W.Q_WANG_RDM, qhist=1)
    d["R_cap"] = 600
    run = oracle.OracleRun(d)
    N = 64
    seen_pairs = seen_omitted = 0
    for i in range(d["K"]):
        if i:
            run.step(i)
        s, _, fam, status = run.state(0)
        assert status == 0
        Ri = len(fam)
        st, pi = run.pairing(0)
        o = run.obs()[0, i]
        h = run.qhist()[0, i]
        c = np.bincount(fam)
        if 2 * c.max() > Ri:
            assert st == 1 and o["nPairs"] == 0 and h.sum() == 0
            seen_omitted += 1
            continue
        seen_pairs += 1
        assert st == 0 and sorted(pi) == list(range(Ri)) and valid(fam, pi)
        # same pairing as rebuilt from the two permutations of this temperature
        p0 = oracle.random_permutation(d["seed"], i, 0, Ri, 0)
        sg = oracle.random_permutation(d["seed"], i, 0, Ri, 1)
        assert np.array_equal(oracle.wang_repair(fam, p0, sg)[1], pi)
        a = s.astype(np.int64).reshape(Ri, 8, 8)
        b = a[pi]
        Q = (a * b).sum(axis=(1, 2))
        ab = a * b
        Ql = (ab * np.roll(ab, -1, axis=2)).sum(axis=(1, 2)) + (ab * np.roll(ab, -1, axis=1)).sum(axis=(1, 2))
        assert o["nPairs"] == Ri
        assert o["sumQ"] == Q.sum() and o["sumAbsQ"] == np.abs(Q).sum() and o["sumQ2"] == (Q * Q).sum()
        assert o["sumQl"] == Ql.sum() and o["sumQl2"] == (Ql * Ql).sum()
        np.testing.assert_array_equal(h, np.bincount((N - Q) // 2, minlength=N + 1))
    assert seen_pairs >= 3 and seen_omitted >= 1
