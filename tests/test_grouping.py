"""GPU grouping, bridges and routing table (Algorithm 2, Sec. IV-B) against
brute force on small cases, planted clusters, and the connection count that
the paper reports for 2,000 GPUs (Sec. V, Fig. 4).  CPU only."""
import itertools

import numpy as np
import pytest

import synth
from paper_2205_07125_amd import HostNetwork
from paper_2205_07125_amd import grouping as gr


def _rand_pg(n, density, seed):
    rng = np.random.default_rng(seed)
    PG = (rng.random((n, n)) < density) * rng.random((n, n))
    np.fill_diagonal(PG, 0.0)
    return PG, np.exp(rng.normal(0.0, 0.3, n))


def _planted(n_groups, s, seed, noise=0.0):
    """Clusters of s GPUs under a random relabelling: strong links inside a
    cluster, optional weak ones across."""
    rng = np.random.default_rng(seed)
    N = n_groups * s
    truth = rng.permutation(np.repeat(np.arange(n_groups), s))
    same = truth[:, None] == truth[None, :]
    PG = np.where(same, 0.5 + 0.5 * rng.random((N, N)), noise * rng.random((N, N)))
    np.fill_diagonal(PG, 0.0)
    return PG, np.ones(N), truth


def _same_partition(a, b):
    """Two labelings describe the same grouping."""
    return len(set(zip(a.tolist(), b.tolist()))) == len(set(a.tolist())) == len(set(b.tolist()))


def test_inter_group_traffic_brute_force():
    PG, WG = _rand_pg(9, 0.6, 1)
    go = np.array([0, 1, 2, 0, 1, 2, 0, 1, 2])
    want = sum(PG[i, j] * WG[i] * WG[j] for i in range(9) for j in range(9) if go[i] != go[j])
    assert gr.inter_group_traffic(PG, WG, go) == pytest.approx(want, rel=1e-12)
    assert gr.inter_group_traffic(PG, WG, np.zeros(9, np.int64)) == 0.0


@pytest.mark.parametrize("seed", range(4))
def test_planted_clusters_recovered(seed):
    PG, WG, truth = _planted(5, 6, seed)
    go = gr.group_gpus(PG, WG, 5, iters=1, seed=seed)
    assert _same_partition(go, truth)
    assert gr.inter_group_traffic(PG, WG, go) == 0.0


@pytest.mark.parametrize("seed", range(6))
def test_best_of_iterations_matches_exhaustive_optimum(seed):
    """8 GPUs in 2 groups of 4, weak noise across planted clusters: the kept
    grouping is the optimum of all 35 balanced splits."""
    PG, WG, truth = _planted(2, 4, seed, noise=0.2)
    best = np.inf
    for first in itertools.combinations(range(1, 8), 3):
        go = np.ones(8, np.int64)
        go[[0, *first]] = 0
        best = min(best, gr.inter_group_traffic(PG, WG, go))
    go = gr.group_gpus(PG, WG, 2, iters=8, seed=seed)
    assert gr.inter_group_traffic(PG, WG, go) == pytest.approx(best, rel=1e-12)
    assert _same_partition(go, truth)


def test_more_iterations_never_worse():
    PG, WG = _rand_pg(60, 0.3, 7)
    first = gr.greedy_groups(PG, WG, 8)
    kept = gr.group_gpus(PG, WG, 8, iters=6, seed=3)
    assert gr.inter_group_traffic(PG, WG, kept) <= gr.inter_group_traffic(PG, WG, first)
    assert np.array_equal(gr.group_gpus(PG, WG, 8, iters=1), first)


@pytest.mark.parametrize("N,n_groups", [(10, 3), (64, 8), (37, 5), (7, 7), (5, 1), (5, 4),
                                        (9, 8), (17, 16)])
def test_groups_cover_and_respect_cap(N, n_groups):
    PG, WG = _rand_pg(N, 0.5, N)
    go = gr.group_gpus(PG, WG, n_groups, iters=3)
    sizes = np.bincount(go, minlength=n_groups)
    # no group left empty, also with equal volumes and a full PG
    full = np.bincount(gr.greedy_groups(np.ones((N, N)) - np.eye(N), np.ones(N), n_groups),
                       minlength=n_groups)
    assert full.min() >= 1 and full.max() <= -(-N // n_groups)
    assert len(sizes) == n_groups and sizes.min() >= 1
    assert sizes.max() <= -(-N // n_groups) and sizes.sum() == N
    with pytest.raises(ValueError):
        gr.greedy_groups(PG, WG, N + 1)


def test_volume_target_closes_a_group():
    """GPU 0 alone carries the mean group volume, so its group closes at one
    member; group 1 then fills to the cap (3 of 6), and the two GPUs left
    join group 0, the only one with room."""
    PG = np.ones((6, 6)) - np.eye(6)
    WG = np.array([5.0, 1, 1, 1, 1, 1])
    assert gr.greedy_groups(PG, WG, 2).tolist() == [0, 1, 1, 1, 0, 0]
    # with equal volumes nothing closes early: two groups of three
    assert np.bincount(gr.greedy_groups(PG, np.ones(6), 2)).tolist() == [3, 3]


def _bridges_ok(PG, WG, go, br):
    n_groups = go.max() + 1
    for g in range(n_groups):
        assert br[g, g] == -1
        members = np.where(go == g)[0]
        roles = [np.count_nonzero(br[g] == m) for m in members]
        assert max(roles) - min(roles) <= 1
        for h in range(n_groups):
            if h != g:
                assert go[br[g, h]] == g


def test_bridges_balanced_and_in_group():
    PG, WG = _rand_pg(50, 0.4, 2)
    go = gr.group_gpus(PG, WG, 9, iters=2)
    _bridges_ok(PG, WG, go, gr.select_bridges(PG, WG, go, balance="roles"))
    with pytest.raises(ValueError):
        gr.select_bridges(PG, WG, go, balance="random")
    with pytest.raises(ValueError):
        gr.select_bridges(PG, WG, np.where(go == 0, go.max() + 1, go))   # group 0 empty


@pytest.mark.parametrize("seed", range(3))
def test_traffic_balanced_bridges_meet_list_scheduling_bound(seed):
    """Largest flow first onto the least loaded member: no bridge carries
    more than the mean load of its group's members plus the largest flow
    (Graham's bound), and the heaviest bridge is no heavier than under
    role balancing on uneven traffic."""
    PG, WG = gr.synthetic_pg(160, 20, 0.9, 0.05, seed=seed, wg_sigma=0.8)
    go = gr.group_gpus(PG, WG, 20, iters=2)
    T = PG * np.outer(WG, WG)
    n_groups = go.max() + 1
    flow = np.array([[T[np.ix_(go == g, go == h)].sum() for h in range(n_groups)]
                     for g in range(n_groups)])
    np.fill_diagonal(flow, 0.0)
    peak = {}
    for balance in ("traffic", "roles"):
        br = gr.select_bridges(PG, WG, go, balance=balance)
        load = np.zeros(len(WG))
        for g in range(n_groups):
            for h in range(n_groups):
                if h != g:
                    assert go[br[g, h]] == g
                    load[br[g, h]] += flow[g, h]
        peak[balance] = load.max()
        if balance == "traffic":
            for g in range(n_groups):
                m = go == g
                assert load[m].max() <= flow[g].sum() / m.sum() + flow[g].max() + 1e-9
    assert peak["traffic"] <= peak["roles"]


def test_bridge_prefers_member_with_traffic():
    """Group {0, 1} sends to group {2, 3} only from GPU 1: GPU 1 bridges."""
    PG = np.zeros((4, 4))
    PG[0, 1] = PG[1, 0] = PG[2, 3] = PG[3, 2] = 1.0
    PG[1, 2] = 0.3
    go = np.array([0, 0, 1, 1])
    br = gr.select_bridges(PG, np.ones(4), go)
    assert br[0, 1] == 1
    assert br[1, 0] in (2, 3)


def test_routing_table_two_hops():
    PG, WG = _rand_pg(40, 0.5, 5)
    go = gr.group_gpus(PG, WG, 6, iters=2)
    br = gr.select_bridges(PG, WG, go)
    TB = gr.routing_table(go, br)
    N = 40
    for i in range(N):
        for j in range(N):
            h = TB[i, j]
            if go[i] == go[j]:
                assert h == j
            elif i == br[go[i], go[j]]:
                assert h == j                        # i is the bridge: it sends directly
            else:
                assert h == br[go[i], go[j]]         # first hop: the group's bridge
                assert go[h] == go[i] and TB[h, j] == j


def test_hops_brute_force():
    PG, WG = _rand_pg(14, 0.5, 11)
    go = gr.group_gpus(PG, WG, 4, iters=2)
    TB = gr.routing_table(go, gr.select_bridges(PG, WG, go))
    want = [set() for _ in range(14)]
    for i in range(14):
        for j in range(14):
            if i != j and PG[i, j] > 0:
                h = TB[i, j]
                want[i].add(h)
                if h != j:
                    want[h].add(j)
    want = [w - {k} for k, w in enumerate(want)]
    H = gr.hop_matrix(PG > 0, TB)
    assert [set(np.nonzero(H[k])[0].tolist()) for k in range(14)] == want
    assert np.array_equal(gr.connections(PG, TB), [len(w) for w in want])
    assert np.array_equal(gr.connections(PG), ((PG > 0).sum(axis=1)))


def test_connections_closed_form_full_exchange():
    """Every pair exchanges traffic: a GPU has s - 1 links in its group and s
    per bridge role, so the mean is s + n_groups - 2."""
    N, s = 48, 6
    PG = np.ones((N, N)) - np.eye(N)
    go = gr.group_gpus(PG, np.ones(N), N // s, iters=1)
    br = gr.select_bridges(PG, np.ones(N), go, balance="roles")
    conn = gr.connections(PG, gr.routing_table(go, br))
    roles = np.array([np.count_nonzero(br == i) for i in range(N)])
    assert np.array_equal(conn, (s - 1) + roles * s)
    assert conn.mean() == s + N // s - 2
    assert gr.connections(PG).tolist() == [N - 1] * N


def test_paper_connection_count_2000_gpus():
    """2,000 GPUs where a GPU reaches 1,552 others on average (Sec. V,
    Fig. 4): groups of the size dense_group_size picks bring the mean down
    to the paper's 88."""
    N = 2000
    rng = np.random.default_rng(2205)
    PG = (rng.random((N, N)) < 1552 / 1999) * rng.random((N, N))
    np.fill_diagonal(PG, 0.0)
    WG = np.exp(rng.normal(0.0, 0.3, N))
    s = gr.dense_group_size(N)
    go = gr.group_gpus(PG, WG, -(-N // s), iters=1)
    TB = gr.routing_table(go, gr.select_bridges(PG, WG, go))
    assert abs(gr.connections(PG).mean() - 1552) < 3
    assert round(gr.connections(PG, TB).mean()) == 88


def test_dense_group_size():
    for n in (1, 2, 9, 100, 2000, 4000):
        s = gr.dense_group_size(n)
        best = min(t + -(-n // t) - 2 for t in range(1, n + 1))
        assert s + -(-n // s) - 2 == best
    assert gr.dense_group_size(2000) in (40, 45, 44, 50)


def test_link_load_brute_force():
    PG, WG = _rand_pg(12, 0.6, 4)
    go = gr.group_gpus(PG, WG, 3, iters=2)
    TB = gr.routing_table(go, gr.select_bridges(PG, WG, go))
    T = PG * np.outer(WG, WG)
    want = np.zeros((12, 12))
    for i in range(12):
        for j in range(12):
            if i != j and T[i, j]:
                h = TB[i, j]
                want[i, h] += T[i, j]
                if h != j:
                    want[h, j] += T[i, j]
    L = gr.link_load(T, TB)
    assert np.allclose(L, want, rtol=1e-12, atol=0)
    # flat exchange: TB = identity routing carries T unchanged
    flat = np.tile(np.arange(12), (12, 1))
    assert np.allclose(gr.link_load(T, flat), T - np.diag(np.diag(T)))


def test_relabel_makes_groups_contiguous():
    go = np.array([2, 0, 1, 0, 2, 1, 1, 2, 0])
    new = gr.relabel(go)
    assert sorted(new.tolist()) == list(range(9))
    assert np.array_equal(new // 3, go)
    assert new[1] < new[3] < new[8]                  # old order kept within a group


def test_partition_graph_matches_synapse_list():
    wl = synth.get_workload("heavy").scaled(1500, k_in=200, vp_set_size=30)
    host = HostNetwork(wl)
    P = wl.n_partitions
    PG, WG = gr.partition_graph(host.part, host.vp_ptr, host.vp_part, P)
    gen = synth.Generator(wl)
    e = gen.edges()
    part = gen.part_map().astype(np.int64)
    src = e["src"].astype(np.int64)
    vp = e["vp"].astype(np.int64)
    remote = vp != part[src]
    pairs = np.unique(np.stack([src[remote], vp[remote]]), axis=1)
    counts = np.zeros((P, P))
    np.add.at(counts, (part[pairs[0]], pairs[1]), 1.0)
    size = np.bincount(part, minlength=P)
    assert np.array_equal(WG, counts.sum(axis=1))
    assert np.allclose(PG, counts / np.maximum(size, 1)[:, None], rtol=0, atol=0)
    go = gr.group_gpus(PG, WG, max(P // wl.gpus_per_node, 1), iters=2)
    assert np.bincount(go).sum() == P


def test_routing_report_consistent():
    PG, WG = _rand_pg(30, 0.5, 9)
    r = gr.routing_report(PG, WG, 5, iters=3, seed=1)
    go, TB = r["group_of"], r["TB"]
    T = PG * np.outer(WG, WG)
    cross = go[:, None] != go[None, :]
    # all cross-group traffic leaves on level-2 hops, from a bridge, once
    assert r["level2_two_level"].sum() == pytest.approx((T * cross).sum(), rel=1e-12)
    assert r["inter_group_traffic"] == pytest.approx((T * cross).sum(), rel=1e-12)
    assert np.allclose(r["level2_flat"], (T * cross).sum(axis=1))
    # only bridges send level-2 traffic
    bridges = set(r["bridge"][r["bridge"] >= 0].tolist())
    assert all(k in bridges for k in np.nonzero(r["level2_two_level"])[0])
    assert r["mean_connections_two_level"] <= r["mean_connections_flat"]


def test_command_line_report(capsys):
    import json
    gr._main(["--gpus", "100", "--reach", "99", "--group-size", "10"])
    out = json.loads(capsys.readouterr().out)
    # every pair connected, groups of 10: s + n_groups - 2 = 18 on average
    assert out["mean_connections_flat"] == 99
    assert out["mean_connections_two_level"] == 18
    assert out["groups"] == 10
