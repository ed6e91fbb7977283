"""links.link_traffic's bookkeeping on hand-made routing buffers (no GPU):
entries per (source partition, destination partition), messages per
(source partition, destination node), the level-1 / level-2 split and the
connection counts."""
import types

import numpy as np
import pytest

from paper_2205_07125_amd.links import link_traffic


class _FakeSim:
    def __init__(self, lists, buckets, P, G):
        self.wl = types.SimpleNamespace(n_partitions=P, gpus_per_node=G,
                                        n_nodes=(P + G - 1) // G)
        self._lists, self._buckets = lists, buckets

    def read_routes(self, which, sources_only=False):
        assert sources_only
        src = self._buckets if which == 2 else self._lists
        return [np.asarray(x, np.uint32) for x in src]


def test_link_traffic_hand_example():
    # 6 neurons, partitions 0,0,1,2,3,3; P = 4 partitions on 2 nodes of 2
    part = np.array([0, 0, 1, 2, 3, 3])
    # neuron 0 (partition 0) reaches partitions 1, 2, 3; neuron 4 (partition 3)
    # reaches partitions 0 and 2
    lists = [[4], [0], [0, 4], [0]]
    buckets = [[0, 4], [0, 4]]          # node 0 = {0, 1}, node 1 = {2, 3}
    got = link_traffic(_FakeSim(lists, buckets, 4, 2), part)
    pm = np.zeros((4, 4), np.int64)
    pm[0, 1] = pm[0, 2] = pm[0, 3] = 1
    pm[3, 0] = pm[3, 2] = 1
    assert np.array_equal(got["partition_matrix"], pm)
    nm = np.zeros((4, 2), np.int64)
    nm[0, 0] = nm[0, 1] = 1
    nm[3, 0] = nm[3, 1] = 1
    assert np.array_equal(got["node_matrix"], nm)
    # partition 0's own node is 0, partition 3's is 1
    assert got["level1"] == 2 and got["level2"] == 2
    assert list(got["connections_flat"]) == [3, 0, 0, 2]
    assert list(got["connections_two_level"]) == [2, 0, 0, 2]
    assert got["max_partition_link"] == 1 and got["max_node_link"] == 1


def test_link_traffic_flat_only():
    part = np.array([0, 1])
    lists = [[1], [0]]
    got = link_traffic(_FakeSim(lists, None, 2, 1), part, two_level=False)
    assert np.array_equal(got["partition_matrix"], np.array([[0, 1], [1, 0]]))
    assert "node_matrix" not in got


def test_bridge_load_hand_example():
    from paper_2205_07125_amd.links import bridge_load
    # 4 partitions on 2 nodes of 2; messages per (source partition, node)
    nm = np.array([[9, 5],      # p0 (node 0): 5 level-2 messages to node 1
                   [0, 3],      # p1 (node 0): 3 to node 1
                   [4, 7],      # p2 (node 1): 4 to node 0
                   [2, 1]])     # p3 (node 1): 2 to node 0
    f = bridge_load(nm, 2, "fixed")
    assert f["bridge"].tolist() == [[-1, 2], [-1, 2], [0, -1], [0, -1]]
    assert f["load"].tolist() == [6, 0, 8, 0] and f["peak"] == 8
    r = bridge_load(nm, 2, "rotate")
    assert r["bridge"].tolist() == [[-1, 2], [-1, 3], [0, -1], [1, -1]]
    assert r["load"].tolist() == [4, 2, 5, 3] and r["peak"] == 5
    b = bridge_load(nm, 2, "balanced")
    assert b["load"].tolist() == [4, 2, 5, 3]
    assert f["connections"].tolist() == [1, 1, 1, 1]


def test_bridge_load_policies_on_random_traffic():
    from paper_2205_07125_amd.links import bridge_load
    rng = np.random.default_rng(5)
    P, G = 40, 8
    nm = rng.poisson(rng.gamma(0.7, 6.0, (P, P // G)))
    own = np.arange(P) // G
    level2 = nm.copy()
    level2[np.arange(P), own] = 0
    res = {pol: bridge_load(nm, G, pol) for pol in ("fixed", "rotate", "balanced")}
    for pol, r in res.items():
        # every level-2 message lands on one member of its destination node
        assert r["load"].sum() == level2.sum()
        br = r["bridge"]
        sent = level2 > 0
        assert np.all((br >= 0) == sent)
        assert np.all(br[sent] // G == np.nonzero(sent)[1])
        assert np.array_equal(r["connections"], sent.sum(axis=1))
    # the fixed bridge takes the whole node's level-2 inflow
    assert res["fixed"]["peak"] == level2.sum(axis=0).max()
    # list-scheduling bound per node for the balanced policy
    load = res["balanced"]["load"]
    for n in range(P // G):
        m = slice(n * G, (n + 1) * G)
        assert load[m].max() <= level2[:, n].sum() / G + level2[:, n].max()
    assert res["balanced"]["peak"] <= res["fixed"]["peak"]
    with pytest.raises(ValueError):
        bridge_load(nm, G, "random")
