"""Pins of the oracle's routing (flat, two-level, expansion): the fan-in
example of Sec. IV-B, invariants computed from the raw synapse arrays with
numpy, and brute force on tiny random graphs.  CPU only."""
import numpy as np
from hypothesis import given, settings
from hypothesis import strategies as st

import oracle
from golden_util import read_golden
from oracle_util import make_sim


def test_fig2_fan_in():
    g = read_golden("fig2_fan_in.txt")
    P, G = g["n_partitions"], g["gpus_per_node"]
    dst = g["destination_partition"]
    # two neurons per partition: neuron 2q lives in partition q
    n = 2 * P
    part = np.repeat(np.arange(P), 2).astype(np.int32)
    srcs = [2 * q for q in g["source_partitions"]]
    edges = [(s, 2 * dst, 1, dst, 0.5) for s in srcs]
    u0 = np.zeros(n, np.float32)
    u0[srcs] = 20.0
    sim = make_sim(n, edges=edges, part=part, u0=u0, n_partitions=P, gpus_per_node=G)
    assert sim.step() == len(srcs)
    flat, xrecv, buckets = sim.recv(0), sim.recv(1), sim.buckets()
    c = sim.counters()
    assert len(flat[dst]) == g["flat_entries_into_destination"]
    assert len({int(part[s]) for s in flat[dst]}) == g["flat_connections_into_destination"]
    assert sum(len(b) for b in buckets) == g["two_level_messages"]
    assert c[oracle.MSG_L1] == g["two_level_level1_messages"]
    assert c[oracle.MSG_L2] == g["two_level_level2_messages"]
    dnode = dst // G
    masks = {int(m[1]) for m in buckets[dnode]}
    assert masks == {g["two_level_mask"]}
    src_nodes = {int(part[m[0]]) // G for m in buckets[dnode]}
    assert len(src_nodes) == g["source_nodes_sending_to_destination_node"]
    assert sorted(xrecv[dst]) == sorted(flat[dst])
    # connections in the paper's sense, from the routed messages: which
    # partition sends to which (the masks of the node buckets), routed by
    # Algorithm 2's table with groups = nodes, where a source reaches another
    # group through its own group's bridge, which forwards to the destination
    from paper_2205_07125_amd import grouping
    dest = np.zeros((P, P), bool)
    for nd, b in enumerate(buckets):
        for m in b:
            s, mask = int(m[0]), int(m[1])
            for bit in range(G):
                if mask >> bit & 1:
                    dest[part[s], G * nd + bit] = True
    group_of = np.arange(P) // G
    TB = grouping.routing_table(group_of, grouping.select_bridges(dest.astype(float), np.ones(P),
                                                                  group_of))
    hops = grouping.hop_matrix(dest, TB)
    assert int(hops[:, dst].sum()) == g["connections_into_destination_after_expansion"]
    # without the table (flat peer-to-peer) every source partition connects to dst
    assert int(dest[:, dst].sum()) == g["flat_connections_into_destination"]
    for p in range(P):
        if p != dst:
            assert len(flat[p]) == 0 and len(xrecv[p]) == 0


def _check_routes(sim, edges, part, G, P):
    """Invariants of one step's routes, computed from the synapse arrays."""
    fired = sim.fired()
    flat, xrecv, buckets = sim.recv(0), sim.recv(1), sim.buckets()
    c = sim.counters()
    src, vp = edges["src"].astype(np.int64), edges["vp"].astype(np.int64)
    remote = vp != part[src]
    # VP(s) and destination nodes per fired source, from numpy unique
    want_flat = {p: [] for p in range(P)}
    want_nodes = 0
    want_buckets = {}
    for s in fired:
        sel = (src == s) & remote
        vps = np.unique(vp[sel])
        for p in vps:
            want_flat[int(p)].append(int(s))
        nodes = np.unique(vps // G)
        want_nodes += len(nodes)
        for nd in nodes:
            bits = vps[vps // G == nd] - G * nd
            mask = 0
            for bit in bits:
                mask |= 1 << int(bit)
            want_buckets.setdefault(int(nd), []).append((mask, int(s)))
    # I1: messages = distinct destination nodes per spike
    assert c[oracle.MSG_L1] + c[oracle.MSG_L2] == want_nodes
    assert sum(len(b) for b in buckets) == want_nodes
    # flat = brute force
    for p in range(P):
        assert sorted(flat[p].tolist()) == sorted(want_flat[p])
    assert c[oracle.FLAT_MSGS] == sum(len(v) for v in want_flat.values())
    # two-level buckets = brute force (mask, src) pairs
    for nd, b in enumerate(buckets):
        got = sorted((int(m[1]), int(m[0])) for m in b)
        assert got == sorted(want_buckets.get(nd, []))
    # I2: expansion reproduces the flat lists as multisets
    for p in range(P):
        assert sorted(xrecv[p].tolist()) == sorted(flat[p].tolist())
    # I4: entries = sum of mask popcounts
    pop = sum(bin(int(m[1])).count("1") for b in buckets for m in b)
    assert pop == c[oracle.RECV_ENTRIES] == sum(len(x) for x in xrecv)
    # I6: masks nonzero, own-partition bit never set, only valid partitions;
    # level split by the source's own node
    l1 = 0
    for nd, b in enumerate(buckets):
        for m in b:
            mask, s = int(m[1]), int(m[0])
            assert mask != 0 and mask < (1 << G)
            for bit in range(G):
                if mask >> bit & 1:
                    assert G * nd + bit < P
                    assert G * nd + bit != part[s]
            l1 += int(part[s]) // G == nd
    assert l1 == c[oracle.MSG_L1]
    # I5: two-level never exceeds flat
    assert want_nodes <= c[oracle.FLAT_MSGS]


@settings(max_examples=60, deadline=None)
@given(data=st.data())
def test_routing_brute_force_random(data):
    # group sizes up to 64: masks of one to 64 bits, including the top bit
    G = data.draw(st.sampled_from([1, 2, 4, 8, 16, 40, 63, 64]))
    P = data.draw(st.integers(1, min(2 * G + 3, 140)))
    n = data.draw(st.integers(max(P, 2), max(P, 2) + 64))
    # contiguous partitions, every partition non-empty
    cuts = sorted(data.draw(st.lists(st.integers(1, n - 1), min_size=P - 1, max_size=P - 1,
                                     unique=True))) if P > 1 else []
    starts = [0] + cuts + [n]
    part = np.zeros(n, np.int32)
    for p in range(P):
        part[starts[p]:starts[p + 1]] = p
    m = data.draw(st.integers(0, 300))
    seed = data.draw(st.integers(0, 2**31))
    rng = np.random.default_rng(seed)
    src = rng.integers(0, n, m)
    tgt = rng.integers(0, n, m)
    ok = src != tgt
    src, tgt = src[ok], tgt[ok]
    delay = rng.integers(1, 11, len(src))
    w = np.where(src % 5 == 4, -2.5, 0.5)
    edges = [(int(a), int(b), int(d), int(part[b]), float(x)) for a, b, d, x in
             zip(src, tgt, delay, w)]
    fire = rng.random(n) < data.draw(st.floats(0.0, 1.0))
    u0 = np.where(fire, 20.0, 0.0).astype(np.float32)
    sim = make_sim(n, edges=edges, part=part, u0=u0, n_partitions=P, gpus_per_node=G)
    sim.step()
    assert np.array_equal(sim.fired(), np.flatnonzero(fire).astype(np.uint32))
    arr = dict(src=np.array([e[0] for e in edges], np.int64),
               vp=np.array([e[3] for e in edges], np.int64))
    _check_routes(sim, arr, part, G, P)


def test_tiny_routes_every_step():
    """tiny_active (8 partitions on 2 nodes of 4, in-degree 100): invariants on
    every step, and the special case of exactly 7 flat entries and 2 two-level
    messages per spike (a source misses one of 8 partitions with probability
    about (7/8)^100)."""
    import synth
    wl = synth.get_workload("tiny_active")
    gen = synth.Generator(wl)
    e = gen.edges()
    part = gen.part_map()
    sim = oracle.Sim(oracle.params_from_workload(wl), e, part, synth.initial_u(wl))
    arr = dict(src=e["src"].astype(np.int64), vp=e["vp"].astype(np.int64))
    total = np.zeros(oracle.NSTAT, np.int64)
    for t in range(120):
        sim.step()
        if t % 10 == 0:
            _check_routes(sim, arr, part, wl.gpus_per_node, wl.n_partitions)
        total += sim.counters().astype(np.int64)
    assert total[oracle.SPIKES] > 500
    assert total[oracle.FLAT_MSGS] == 7 * total[oracle.SPIKES]
    assert total[oracle.MSG_L1] == total[oracle.SPIKES]
    assert total[oracle.MSG_L2] == total[oracle.SPIKES]
