"""k-means over a grid of candidate block counts (oracle side).

The paper maps the embedding to a partition with KMeans (Sec. II, graph
embedding definition; Alg. 1 runs KMeans with K = 2 for T iterations,
Sec. III-C).  It fixes neither the initialisation, the stopping rule, ties nor
empty clusters.  Readings used here (and on the GPU side):

Seeding: k-means++ (D^2 sampling, Arthur & Vassilvitskii 2007) realised as an
exponential race (Efraimidis & Spirakis 2006): with weights w_i (1 before the
first pick, afterwards the squared distance to the nearest pick), pick
t = argmin_{i: w_i > 0} E_{t,i} / w_i with E_{t,i} = -ln u and u the first
Philox word of key (seed, 0x20), counter (i, t, 0, 0); ties go to the lowest i;
if every w_i is 0 the lowest unpicked index is taken.  Picks are nested: the
candidate with K blocks starts from the first K picks.  The ratio is formed in
FP64.

Lloyd: a_i = argmin_k ||z_i - c_k||^2 (ties to the lowest k); stop when the
assignment equals the previous one (from the second assignment on) or after
T_max assignments; c_k = mean of its members, an empty cluster keeps its
centre.  A converged candidate is a fixed point of the iteration.

Pinned in ``tests/test_oracle_kmeans.py``: fixed-point invariants, agreement
with scikit-learn's Lloyd from the same initial centres, brute force on tiny
inputs, and D^2 pick frequencies of the race.
"""
import numpy as np

from . import fmath, philox


def race_exponentials(seed, n, t):
    """E_{t,i} = -ln u for i = 0..n-1 at pick t (FP64)."""
    ctr = np.zeros((n, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(n, dtype=np.uint64)
    ctr[:, 1] = np.uint64(t)
    blk = philox.philox4x64(ctr, np.array([seed, philox.STREAM_RACE], dtype=np.uint64))
    return -fmath.ln(fmath.uniform52(blk[:, 0]))


def seed_picks(z, k_max, seed):
    """Nested k-means++ picks p_0..p_{k_max-1} by the exponential race."""
    z = np.asarray(z, dtype=np.float64)
    n = z.shape[0]
    if k_max > n:
        raise ValueError("k_max exceeds the number of points")
    w = np.ones(n, dtype=np.float64)
    picked = np.zeros(n, dtype=bool)
    picks = []
    for t in range(k_max):
        e = race_exponentials(seed, n, t)
        pos = w > 0
        if np.any(pos):
            ratio = np.full(n, np.inf)
            ratio[pos] = e[pos] / w[pos]
            p = int(np.argmin(ratio))       # first index of the minimum
        else:
            p = int(np.flatnonzero(~picked)[0])
        picks.append(p)
        picked[p] = True
        diff = z - z[p]
        dist = np.sum(diff * diff, axis=1)
        w = dist if t == 0 else np.minimum(w, dist)
    return np.array(picks, dtype=np.int64)


def sq_distances(z, c):
    """||z_i - c_k||^2 for all i, k (FP64)."""
    zz = np.sum(z * z, axis=1)[:, None]
    cc = np.sum(c * c, axis=1)[None, :]
    return zz - 2.0 * (z @ c.T) + cc


def lloyd(z, centres, t_max=100):
    """Lloyd's iteration from the given centres.

    Returns (labels int64 [n], centres [K, d], assignments performed)."""
    z = np.asarray(z, dtype=np.float64)
    c = np.array(centres, dtype=np.float64, copy=True)
    k = c.shape[0]
    prev = None
    it = 0
    a = None
    for it in range(1, t_max + 1):
        a = np.argmin(sq_distances(z, c), axis=1)
        if prev is not None and np.array_equal(a, prev):
            break
        for r in range(k):
            members = a == r
            if np.any(members):
                c[r] = z[members].mean(axis=0)
        prev = a
    return a.astype(np.int64), c, it


def kgrid(k_min, k_max, k_step=1):
    return list(range(k_min, k_max + 1, k_step))


def multi_k(z, ks, seed, t_max=100):
    """Run Lloyd for every candidate K in ks from the nested picks.

    Returns dict(picks, labels [n, len(ks)] int64, iters [len(ks)])."""
    picks = seed_picks(z, max(ks), seed)
    labels = np.zeros((z.shape[0], len(ks)), dtype=np.int64)
    iters = np.zeros(len(ks), dtype=np.int64)
    for j, k in enumerate(ks):
        a, _, it = lloyd(z, np.asarray(z, np.float64)[picks[:k]], t_max)
        labels[:, j] = a
        iters[j] = it
    return {"picks": picks, "labels": labels, "iters": iters}
