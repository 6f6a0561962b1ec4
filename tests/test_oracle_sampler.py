"""Pins of the fast SBM sampler (Sec. IV, Alg. 2): edge frequencies over many
seeds against 1 - exp(-lambda_ij) pair by pair (binomial bound), expected edge
counts against the closed form sum (1 - exp(-lambda)), degenerate
intensities, agreement in distribution with a direct Bernoulli sampler, and a
valid symmetric loop-free CSR."""
import numpy as np
import pytest

from oracle import graph as ograph
from oracle import sbm_sample


def tiny_model():
    theta = np.array([0.5, 1.0, 1.5, 0.8, 1.2, 0.7, 1.1])
    blocks = np.array([0, 1, 0, 1, 0, 1, 1])
    omega = np.array([[0.9, 0.15], [0.15, 0.6]])
    return theta, blocks, omega


def lam_matrix(theta, blocks, omega):
    return np.outer(theta, theta) * omega[blocks][:, blocks]


def test_pair_frequencies_match_model():
    theta, blocks, omega = tiny_model()
    n = theta.size
    p = 1.0 - np.exp(-lam_matrix(theta, blocks, omega))
    trials = 3000
    hits = np.zeros((n, n))
    for seed in range(trials):
        a, b = sbm_sample.sample_edges(theta, blocks, omega, seed)
        assert np.all(a != b)
        i, j = np.minimum(a, b), np.maximum(a, b)
        assert np.unique(i * n + j).size == i.size          # each pair at most once
        hits[i, j] += 1
    iu = np.triu_indices(n, 1)
    freq = hits[iu] / trials
    sd = np.sqrt(p[iu] * (1 - p[iu]) / trials)
    assert np.all(np.abs(freq - p[iu]) < 4.5 * sd + 1e-12), np.max(np.abs(freq - p[iu]) / sd)
    assert np.all(np.tril(hits) == 0)


def test_expected_edge_count_closed_form():
    rng = np.random.default_rng(4)
    n, k = 300, 4
    blocks = rng.integers(0, k, n)
    theta = rng.uniform(0.2, 2.0, n)
    omega = np.full((k, k), 0.002) + np.eye(k) * 0.02
    lam = lam_matrix(theta, blocks, omega)
    expect = np.sum(1.0 - np.exp(-lam[np.triu_indices(n, 1)]))
    counts = [sbm_sample.sample_edges(theta, blocks, omega, s)[0].size for s in range(200)]
    var = np.sum((1 - np.exp(-lam[np.triu_indices(n, 1)])) * np.exp(-lam[np.triu_indices(n, 1)]))
    assert abs(np.mean(counts) - expect) < 4.0 * np.sqrt(var / 200)


def test_degenerate_intensities():
    theta, blocks, omega = tiny_model()
    a, _ = sbm_sample.sample_edges(theta, blocks, np.zeros_like(omega), 1)
    assert a.size == 0
    # overwhelming intensity: every pair is joined
    a, b = sbm_sample.sample_edges(theta, blocks, np.full_like(omega, 1e6), 1)
    n = theta.size
    assert a.size == n * (n - 1) // 2


def test_agrees_with_direct_bernoulli_in_distribution():
    """Degree distribution of the jump sampler against a per-pair Bernoulli
    (1 - exp(-lambda)) sampler: two-sample chi-square on pooled degrees."""
    from scipy import stats
    rng = np.random.default_rng(7)
    n, k = 200, 3
    blocks = rng.integers(0, k, n)
    theta = rng.uniform(0.3, 1.7, n)
    omega = np.full((k, k), 0.004) + np.eye(k) * 0.05
    p = 1 - np.exp(-lam_matrix(theta, blocks, omega))
    iu = np.triu_indices(n, 1)
    d_jump, d_direct = [], []
    for s in range(150):
        a, b = sbm_sample.sample_edges(theta, blocks, omega, s)
        d_jump.append(np.bincount(np.concatenate([a, b]), minlength=n))
        keep = rng.random(iu[0].size) < p[iu]
        d_direct.append(np.bincount(np.concatenate([iu[0][keep], iu[1][keep]]), minlength=n))
    dj, dd = np.concatenate(d_jump), np.concatenate(d_direct)
    edges = np.arange(0, max(dj.max(), dd.max()) + 2)
    hj, _ = np.histogram(dj, edges)
    hd, _ = np.histogram(dd, edges)
    keep = (hj + hd) >= 10
    _, pval, _, _ = stats.chi2_contingency(np.vstack([hj[keep], hd[keep]]))
    assert pval > 1e-3
    # per-node mean degrees agree with the model
    md = np.mean(d_jump, axis=0)
    ed = p.sum(axis=1) - np.diag(p)
    assert np.abs(md - ed).max() < 5 * np.sqrt(ed.max() / 150) + 0.5


def test_csr_is_valid():
    rng = np.random.default_rng(2)
    n, k = 500, 5
    blocks = rng.integers(0, k, n)
    theta = rng.uniform(0.5, 3.0, n)
    omega = np.full((k, k), 0.003) + np.eye(k) * 0.03
    rp, ci = sbm_sample.sample_csr(theta, blocks, omega, 11)
    ograph.validate_csr(rp.astype(np.int32), ci.astype(np.int32), n)
    # deterministic in the seed
    rp2, ci2 = sbm_sample.sample_csr(theta, blocks, omega, 11)
    assert np.array_equal(rp, rp2) and np.array_equal(ci, ci2)


def test_row_form_equals_table_form():
    """The scalar per-row form gives, row by row, the table form's edges
    (models with an empty block, a one-node block and a strong diagonal)."""
    rng = np.random.default_rng(5)
    n, k = 120, 5
    blocks = rng.integers(0, k, n)
    blocks[blocks == 3] = 1                       # block 3 empty
    blocks[7] = 4
    blocks[blocks == 4] = 2
    blocks[7] = 4                                 # block 4 = one node
    theta = rng.uniform(0.2, 2.5, n)
    omega = np.full((k, k), 0.02) + np.eye(k) * 0.3
    members = sbm_sample.block_members(blocks, k)
    pref = [sbm_sample.prefix(theta, m) for m in members]
    for seed in (0, 9):
        a, b = sbm_sample.sample_edges(theta, blocks, omega, seed)
        got_a, got_b = [], []
        for r in range(k):
            for s in range(r, k):
                if members[r].size == 0 or members[s].size == 0:
                    continue
                for x in range(members[r].size):
                    cols = sbm_sample.row_edges(theta, members, pref, omega, r, s, x, seed)
                    got_a += [int(members[r][x])] * len(cols)
                    got_b += cols
        # the table form emits jump by jump across rows; compare as edge sets
        assert sorted(zip(a.tolist(), b.tolist())) == sorted(zip(got_a, got_b))
        assert len(got_a) == a.size
