"""Pins of the k-means oracle: Lloyd fixed-point invariants, scikit-learn's
Lloyd from the same initial centres, brute force on tiny inputs, and the D^2
law of the exponential-race seeding."""
import itertools

import numpy as np
import pytest
from scipy import stats

from oracle import gcn, kmeans, projection


@pytest.fixture(scope="module")
def emb(small_graph):
    g, m = small_graph
    y = projection.project(g.row_ptr, g.col_idx, g.n, projection.NCUT, 64, 3, 0)
    return gcn.embed(g.row_ptr, g.col_idx, g.n, y, [64, 64], 0)


def test_lloyd_fixed_point(emb):
    picks = kmeans.seed_picks(emb, 12, 0)
    for k in (2, 5, 11, 12):
        a, c, it = kmeans.lloyd(emb, emb[picks[:k]], 100)
        assert it < 100
        d = kmeans.sq_distances(emb, c)
        # every point is at (one of) its nearest centres, lowest index on ties
        assert np.array_equal(a, np.argmin(d, axis=1))
        for r in range(k):
            if np.any(a == r):
                np.testing.assert_allclose(c[r], emb[a == r].mean(0), rtol=1e-12, atol=1e-14)


def test_lloyd_matches_sklearn(emb):
    from sklearn.cluster import KMeans
    picks = kmeans.seed_picks(emb, 20, 1)
    for k in (3, 8, 20):
        init = emb[picks[:k]]
        a, c, _ = kmeans.lloyd(emb, init, 300)
        km = KMeans(n_clusters=k, init=init, n_init=1, algorithm="lloyd", tol=0.0,
                    max_iter=300).fit(emb)
        assert np.array_equal(a, km.labels_)


def _objective(z, a, k):
    tot = 0.0
    for r in range(k):
        if np.any(a == r):
            m = z[a == r].mean(0)
            tot += ((z[a == r] - m) ** 2).sum()
    return tot


def test_lloyd_vs_brute_force():
    rng = np.random.default_rng(0)
    # separated planted points: Lloyd from k-means++ reaches the optimum
    cen = np.array([[0, 0], [10, 0], [0, 10]], float)
    z = np.concatenate([c + 0.3 * rng.standard_normal((3, 2)) for c in cen])
    best = min(_objective(z, np.array(a), 3) for a in itertools.product(range(3), repeat=9)
               if len(set(a)) == 3)
    picks = kmeans.seed_picks(z, 3, 4)
    a, _, _ = kmeans.lloyd(z, z[picks], 100)
    assert abs(_objective(z, a, 3) - best) < 1e-12
    # random points: Lloyd's local optimum is never better than brute force
    z = rng.standard_normal((8, 2))
    best = min(_objective(z, np.array(a), 2) for a in itertools.product(range(2), repeat=8))
    for s in range(5):
        picks = kmeans.seed_picks(z, 2, s)
        a, _, _ = kmeans.lloyd(z, z[picks], 100)
        assert _objective(z, a, 2) >= best - 1e-12


def test_race_first_pick_uniform_and_d2_law():
    # first pick: argmin of n iid exponentials -> uniform over points
    n, seeds = 5, 8000
    z = np.array([[0.0], [1.0], [3.0], [3.5], [7.0]])
    first = np.zeros(n)
    second = np.zeros(n)
    cond = np.zeros(n)
    for s in range(seeds):
        p = kmeans.seed_picks(z, 2, s)
        first[p[0]] += 1
        if p[0] == 0:
            second[p[1]] += 1
            cond[0] += 1
    assert stats.chisquare(first).pvalue > 1e-4
    # given first pick 0, second pick ~ D^2 = squared distance to point 0
    w = (z[:, 0] - z[0, 0]) ** 2
    expect = cond[0] * w / w.sum()
    mask = expect > 0
    assert second[0] == 0
    assert stats.chisquare(second[mask], expect[mask]).pvalue > 1e-4


def test_race_exponentials_from_philox():
    e = kmeans.race_exponentials(0, 100000, 3)
    assert np.all(e > 0)
    assert stats.kstest(e, "expon").pvalue > 1e-4


def test_picks_distinct_and_duplicates():
    z = np.array([[0.0, 0], [0, 0], [1, 0], [1, 0], [2, 2]])
    p = kmeans.seed_picks(z, 5, 0)
    assert len(set(p.tolist())) == 5        # zero-weight fallback picks unpicked points
    p3 = kmeans.seed_picks(z, 3, 0)
    # the first three picks land on three distinct locations
    assert len({tuple(z[i]) for i in p3}) == 3


def test_multi_k_nested(emb):
    out = kmeans.multi_k(emb, [2, 3, 7], 5, 100)
    assert out["labels"].shape == (emb.shape[0], 3)
    for j, k in enumerate([2, 3, 7]):
        assert out["labels"][:, j].max() < k
