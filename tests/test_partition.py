"""Neuron -> GPU partitioning (Algorithm 1, Sec. IV-A) against brute force on
small cases, planted clusters, its balance bound and closed forms of the
GPU graph it hands to Algorithm 2.  CPU only."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2205_07125_amd import grouping as gr
from paper_2205_07125_amd import partition as pt


def _rand_p(M, density, seed):
    rng = np.random.default_rng(seed)
    P = (rng.random((M, M)) < density) * rng.random((M, M))
    np.fill_diagonal(P, 0.0)
    return P, np.exp(rng.normal(0.0, 0.5, M))


def _planted(n_clusters, s, seed, noise=0.0):
    rng = np.random.default_rng(seed)
    M = n_clusters * s
    truth = rng.permutation(np.repeat(np.arange(n_clusters), s))
    same = truth[:, None] == truth[None, :]
    P = np.where(same, 0.5 + 0.5 * rng.random((M, M)), noise * rng.random((M, M)))
    np.fill_diagonal(P, 0.0)
    return P, np.ones(M), truth


def _same_partition(a, b):
    return len(set(zip(a.tolist(), b.tolist()))) == len(set(a.tolist())) == len(set(b.tolist()))


def test_cut_and_gpu_traffic_brute_force():
    P, W = _rand_p(11, 0.5, 3)
    pm = np.array([0, 1, 2, 0, 1, 2, 0, 1, 2, 0, 1])
    want = np.zeros(3)
    for i in range(11):
        for j in range(11):
            if pm[i] != pm[j]:
                want[pm[i]] += P[i, j] * W[i] * W[j]
    assert pt.cut_traffic(P, W, pm) == pytest.approx(want.sum(), rel=1e-12)
    assert np.allclose(pt.gpu_traffic(P, W, pm, 3), want, rtol=1e-12, atol=0)
    assert pt.cut_traffic(P, W, np.zeros(11, np.int64)) == 0.0


@pytest.mark.parametrize("seed", range(4))
def test_planted_clusters_recovered(seed):
    P, W, truth = _planted(4, 6, seed)
    pm = pt.partition_neurons(P, W, 4, iters=16, seed=seed)
    assert _same_partition(pm, truth)
    assert pt.cut_traffic(P, W, pm) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_matches_exhaustive_optimum(seed):
    """8 neurons on 2 GPUs of equal weight, planted clusters with weak noise
    across: the kept map is the best of all 35 balanced splits."""
    P, W, truth = _planted(2, 4, seed, noise=0.2)
    best = np.inf
    for first in itertools.combinations(range(1, 8), 3):
        pm = np.ones(8, np.int64)
        pm[[0, *first]] = 0
        best = min(best, pt.cut_traffic(P, W, pm))
    pm = pt.partition_neurons(P, W, 2, iters=8, seed=seed)
    assert np.bincount(pm).tolist() == [4, 4]
    assert pt.cut_traffic(P, W, pm) == pytest.approx(best, rel=1e-12)


@pytest.mark.parametrize("M,N,seed", [(50, 4, 0), (200, 7, 1), (31, 31, 2), (40, 1, 3)])
def test_balance_bound_and_cover(M, N, seed):
    P, W = _rand_p(M, 0.1, seed)
    pm = pt.partition_neurons(P, W, N, iters=2, seed=seed)
    assert pm.min() == 0 and pm.max() == N - 1 and len(pm) == M
    load = np.bincount(pm, weights=W, minlength=N)
    assert np.all(load < W.sum() / N + W.max())
    assert load.sum() == pytest.approx(W.sum(), rel=1e-12)


def test_beats_random_on_clustered_input():
    P, W = pt.synthetic_neurons(3000, 12, 15, 3, seed=4)
    N = 6
    pm = pt.partition_neurons(P, W, N, iters=2, seed=0)
    rnd = np.random.default_rng(0).permutation(np.arange(3000) % N)
    assert pt.cut_traffic(P, W, pm) < 0.6 * pt.cut_traffic(P, W, rnd)
    assert pt.gpu_traffic(P, W, pm, N).max() < pt.gpu_traffic(P, W, rnd, N).max()


def test_sparse_and_dense_inputs_agree():
    P, W = _rand_p(60, 0.2, 5)
    seeds = np.array([3, 17, 42])
    a = pt.greedy_pass(P, W, 3, seeds)
    b = pt.greedy_pass(sp.csr_matrix(P), W, 3, seeds)
    assert np.array_equal(a, b)
    assert np.array_equal(pt.partition_neurons(P, W, 3, iters=3, seed=1),
                          pt.partition_neurons(sp.csr_matrix(P), W, 3, iters=3, seed=1))


def test_more_passes_never_worse():
    P, W = pt.synthetic_neurons(800, 6, 10, 4, seed=6)
    one = pt.partition_neurons(P, W, 4, iters=1, seed=2)
    many = pt.partition_neurons(P, W, 4, iters=6, seed=2)
    assert pt.cut_traffic(P, W, many) <= pt.cut_traffic(P, W, one)


def test_bad_arguments():
    P, W = _rand_p(5, 0.5, 0)
    with pytest.raises(ValueError):
        pt.greedy_pass(P, W, 2, np.array([1, 1]))
    with pytest.raises(ValueError):
        pt.greedy_pass(P, W, 6, np.arange(6))


def test_gpu_graph_closed_form_constant_p():
    """P = c for every pair: PG[g, h] = c off the diagonal, whatever the
    map and the weights."""
    M, c = 30, 0.375
    P = np.full((M, M), c)
    np.fill_diagonal(P, 0.0)
    W = np.exp(np.random.default_rng(1).normal(0, 0.5, M))
    pm = np.random.default_rng(2).permutation(np.arange(M) % 4)
    PG, WG = pt.gpu_graph(P, W, pm, 4)
    assert np.allclose(PG[~np.eye(4, dtype=bool)], c, rtol=1e-12, atol=0)
    assert np.all(np.diag(PG) == 0.0)
    assert np.allclose(WG, np.bincount(pm, weights=W))


def test_gpu_graph_feeds_algorithm_2():
    """Algorithm 2's objective on PG, WG equals the neuron traffic between
    GPUs of different groups, counted pair by pair."""
    P, W = _rand_p(40, 0.3, 8)
    pm = pt.partition_neurons(P, W, 8, iters=2, seed=0)
    PG, WG = pt.gpu_graph(P, W, pm, 8)
    assert np.all((PG >= 0) & (PG <= 1))
    go = gr.group_gpus(PG, WG, 3, iters=2)
    want = sum(P[i, j] * W[i] * W[j] for i in range(40) for j in range(40)
               if go[pm[i]] != go[pm[j]])
    assert gr.inter_group_traffic(PG, WG, go) == pytest.approx(want, rel=1e-12)


def test_plan_recovers_two_levels_of_structure():
    """Neurons in 12 clusters of 10, clusters in 4 super-clusters of 3:
    strong links inside a cluster, weaker ones inside a super-cluster, none
    across.  Algorithm 1 puts each cluster on one GPU, Algorithm 2 puts each
    super-cluster's GPUs in one group, so no traffic crosses groups and every
    GPU talks only to its own group."""
    rng = np.random.default_rng(11)
    n_cl, per, sup = 12, 10, 3
    M = n_cl * per
    perm = rng.permutation(M)
    cluster = np.repeat(np.arange(n_cl), per)[perm]
    group = cluster // sup
    same_c = cluster[:, None] == cluster[None, :]
    same_g = group[:, None] == group[None, :]
    P = np.where(same_c, 0.9, np.where(same_g, 0.05, 0.0)) * (0.5 + 0.5 * rng.random((M, M)))
    np.fill_diagonal(P, 0.0)
    W = np.ones(M)
    r = pt.plan(sp.csr_matrix(P), W, n_cl, n_cl // sup, iters=16, seed=3)
    assert _same_partition(r["PM"], cluster)
    assert _same_partition(r["group_of"][r["PM"]], group)
    assert r["inter_group_traffic"] == 0.0
    # flat: a GPU reaches the other two GPUs of its super-cluster; two-level:
    # the same two, inside its group, and nothing else
    assert np.all(r["connections_flat"] == sup - 1)
    assert np.all(r["connections_two_level"] == sup - 1)
    assert r["cut_traffic"] == pytest.approx(r["gpu_traffic"].sum(), rel=1e-12)
    assert r["peak_level2_two_level"] == 0.0


def test_spread_seeds_one_per_separate_cluster():
    """Clusters with no links between them: the first seeds fall in distinct
    clusters, the heaviest neuron first."""
    rng = np.random.default_rng(4)
    cl = rng.permutation(np.repeat(np.arange(7), 9))
    P = np.where(cl[:, None] == cl[None, :], rng.random((63, 63)), 0.0)
    np.fill_diagonal(P, 0.0)
    W = rng.random(63)
    seeds = pt.spread_seeds(pt._sym_csr(P), W, 7)
    assert seeds[0] == int(np.argmax(W))
    assert len(set(cl[seeds].tolist())) == 7
    assert len(set(seeds.tolist())) == 7


def test_spread_seeds_sparse_separate_clusters():
    """Seven disjoint sparse clusters (about five in-cluster links per
    neuron, so most neurons have no direct link to a seed): still one seed in
    each cluster before any cluster gets a second."""
    P, W = pt.synthetic_neurons(700, 7, 5.0, 0.0, seed=6)
    A = pt._sym_csr(P)
    from scipy.sparse.csgraph import connected_components
    n_comp, comp = connected_components(A, directed=False)
    seeds = pt.spread_seeds(A, W, n_comp)
    assert len(set(comp[seeds].tolist())) == n_comp
    # with more seeds than components, the extra ones go to the farthest neurons
    more = pt.spread_seeds(A, W, n_comp + 3)
    assert np.array_equal(more[:n_comp], seeds)
    assert len(set(more.tolist())) == n_comp + 3


def test_device_layout_contiguous_ranges():
    rng = np.random.default_rng(8)
    M, N, G = 200, 12, 4
    pm = rng.integers(0, N, M)
    group_of = rng.permutation(np.repeat(np.arange(N // G), G))
    lay = pt.device_layout(pm, group_of, G)
    q = lay["partition_id"][pm]
    nid, st = lay["neuron_id"], lay["starts"]
    assert sorted(nid.tolist()) == list(range(M))
    assert sorted(lay["partition_id"].tolist()) == list(range(N))
    assert np.all((st[q] <= nid) & (nid < st[q + 1]))
    assert np.array_equal(np.diff(st), np.bincount(q, minlength=N))
    assert np.array_equal(lay["partition_id"] // G, group_of)      # node = group
    # old order kept inside a partition
    for p in range(N):
        ids = np.where(q == p)[0]
        assert np.all(np.diff(nid[ids]) == 1)
    with pytest.raises(ValueError):
        pt.device_layout(pm, np.array([0] * 5 + [1] * 7), G)


def _dense_greedy_pass(P, W, n_gpus, seeds):
    """The pass with a dense GPUs x neurons affinity array and argmax (lowest
    id among ties): the plain form the sparse frontier must reproduce."""
    A = pt._sym_csr(P)
    W = np.asarray(W, np.float64)
    M = len(W)
    target = W.sum() / n_gpus
    pm = np.full(M, -1, np.int64)
    load = np.zeros(n_gpus)
    aff = np.zeros((n_gpus, M))
    free = np.ones(M, bool)

    def place(i, j):
        pm[j] = i
        free[j] = False
        load[i] += W[j]
        lo, hi = A.indptr[j], A.indptr[j + 1]
        aff[i, A.indices[lo:hi]] += A.data[lo:hi]
        aff[:, j] = -np.inf

    for i, j in enumerate(seeds):
        place(i, int(j))
    n_free = M - n_gpus
    while n_free:
        moved = False
        for i in range(n_gpus):
            if not n_free:
                break
            if load[i] >= target:
                continue
            place(i, int(np.argmax(aff[i])))
            n_free -= 1
            moved = True
        if not moved:
            break
    for j in np.where(free)[0][np.argsort(-W[free], kind="stable")]:
        place(int(np.argmin(load)), int(j))
    return pm


@pytest.mark.parametrize("M,N,density,seed", [(40, 3, 0.1, 0), (120, 7, 0.03, 1),
                                              (300, 16, 0.01, 2), (200, 5, 0.0, 3)])
def test_sparse_frontier_equals_dense_argmax(M, N, density, seed):
    """The heap frontier picks what the dense argmax picks, ties and
    neurons without links to a GPU's members (lowest free id) included."""
    P, W = _rand_p(M, density, seed)
    rng = np.random.default_rng(seed + 10)
    seeds = rng.choice(M, N, replace=False)
    assert np.array_equal(pt.greedy_pass(sp.csr_matrix(P), W, N, seeds),
                          _dense_greedy_pass(P, W, N, seeds))


def test_pass_memory_stays_sparse():
    """100,000 neurons on 1,000 GPUs (a dense GPUs x neurons array would take
    800 MB): the pass allocates O(synapses + neurons)."""
    import tracemalloc
    M, N, deg = 100_000, 1_000, 8
    rng = np.random.default_rng(5)
    rows = np.repeat(np.arange(M), deg)
    cols = rng.integers(0, M, M * deg)
    P = sp.csr_matrix((rng.random(M * deg), (rows, cols)), shape=(M, M))
    W = np.ones(M)
    A = pt._sym_csr(P)
    seeds = rng.choice(M, N, replace=False)
    tracemalloc.start()
    pm = pt.greedy_pass(P, W, N, seeds, A=A)
    peak = tracemalloc.get_traced_memory()[1]
    tracemalloc.stop()
    assert peak < 200e6
    assert np.all(pm >= 0) and np.bincount(pm, minlength=N).max() <= M // N + 1
