"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by
element on the same seeded inputs: fired ids, routing buffers (as sorted
multisets per bucket / list), per-step counters, and the full state (u, ref,
delay ring) bit-exactly; the FP64 trajectory within 1e-4 mV."""
import numpy as np
import pytest

import oracle
import synth
from paper_2205_07125_amd._abi import ENTRY_SRC_BITS

pytestmark = pytest.mark.gpu

ROUTE_BOTH = 2
ROUTE_TWO_LEVEL = 0
ROUTE_FLAT = 1

# oracle counter order -> device counter order (both list the same 7 counters)
STAT_MAP = [oracle.SPIKES, oracle.LOCAL_EVENTS, oracle.REMOTE_EVENTS, oracle.MSG_L1,
            oracle.MSG_L2, oracle.FLAT_MSGS, oracle.RECV_ENTRIES]


def _pair(wl, part_map=None, **simkw):
    from paper_2205_07125_amd import HostNetwork, Simulation
    print(f"[gpu] building {wl.name} N={wl.n_neurons} K={wl.k_in} P={wl.n_partitions} "
          f"G={wl.gpus_per_node}", flush=True)
    sim = Simulation(wl, host=HostNetwork(wl, part_map=part_map), **simkw)
    orc = oracle.sim_for_workload(wl, part_map=part_map)
    return sim, orc


def _same_state(sim, orc, where):
    g = sim.state()
    o = orc.state()
    assert np.array_equal(g["u"].view(np.uint32), o["u"].view(np.uint32)), f"u differs at {where}"
    assert np.array_equal(g["ref"], o["ref"]), f"ref differs at {where}"
    assert np.array_equal(g["ring"].view(np.uint32), o["ring"].view(np.uint32)), \
        f"ring differs at {where}"
    return g, o


def _same_routes(sim, orc, wl, where, mode=ROUTE_BOTH):
    """The buffers the route mode fills: flat lists (flat, both), expanded
    lists and node buckets (two-level, both)."""
    flat = mode != ROUTE_TWO_LEVEL
    two = mode != ROUTE_FLAT
    src_mask = np.uint64((1 << ENTRY_SRC_BITS) - 1)
    host = sim.host
    lists = []
    if flat:
        lists.append(("flat", sim.read_routes(0), orc.recv(0)))
    if two:
        lists.append(("expanded", sim.read_routes(1), orc.recv(1)))
    for kind, got, want in lists:
        for p in range(wl.n_partitions):
            g = (got[p] & src_mask).astype(np.uint32)
            assert np.array_equal(np.sort(g), np.sort(want[p])), f"{kind} {p} at {where}"
            # the pair index each entry carries belongs to its source and names p
            if len(got[p]) and host is not None:
                s = (got[p] & src_mask).astype(np.int64)
                j = (got[p] >> np.uint64(ENTRY_SRC_BITS)).astype(np.int64)
                assert np.all(j >= host.vp_ptr[s]) and np.all(j < host.vp_ptr[s + 1])
                assert np.all(host.vp_part[j] == p)
    if two:
        b_g, b_o = sim.read_routes(2), orc.buckets()
        for n in range(wl.n_nodes):
            # (source, mask) multisets; device messages also carry the pair
            # index of the node's first destination above bit 32
            src = b_g[n][:, 0] & np.uint64(0xFFFFFFFF)
            g = sorted(zip(src.tolist(), b_g[n][:, 1].tolist()))
            assert g == sorted(map(tuple, b_o[n].tolist())), f"bucket {n} at {where}"
            if len(src) and host is not None:
                # the pair index is s's first destination in node n
                s_ = src.astype(np.int64)
                j = (b_g[n][:, 0] >> np.uint64(32)).astype(np.int64)
                assert np.all(j >= host.vp_ptr[s_]) and np.all(j < host.vp_ptr[s_ + 1])
                G = wl.gpus_per_node
                assert np.all(host.vp_part[j] // G == n)
                first = (j == host.vp_ptr[s_]) | (host.vp_part[np.maximum(j - 1, 0)] // G != n)
                assert np.all(first)


def _lockstep(wl, n_steps, route_every, state_every, mode=ROUTE_BOTH, fused=False,
              fp64_bound=1e-4, part_map=None, tile_neurons=0):
    """fused: each step as snn_step_route + snn_deliver (two-level routing in
    the update kernel) instead of snn_step, snn_route, snn_deliver.
    fp64_bound: largest |u - u_fp64| allowed (mV); None reports it only.
    part_map: explicit neuron -> partition map of the network.
    tile_neurons: neurons per tile (0: the library's default)."""
    sim, orc = _pair(wl, part_map=part_map, log_steps=n_steps, tile_neurons=tile_neurons)
    stats_o = np.zeros((n_steps, 7), np.uint64)
    fired_o = []
    for t in range(n_steps):
        if fused:
            sim.step_route(mode)
            sim.deliver()
        else:
            sim.full_step(mode)
        orc.step()
        fired_o.append(orc.fired())
        stats_o[t] = orc.counters()[STAT_MAP]
        if route_every and t % route_every == 0:
            _same_routes(sim, orc, wl, f"step {t}", mode)
        if state_every and (t + 1) % state_every == 0:
            _same_state(sim, orc, f"after step {t}")
    ids, counts = sim.read_spikes(0, n_steps)
    assert np.array_equal(counts, np.array([len(f) for f in fired_o], np.uint32))
    assert np.array_equal(ids, np.concatenate(fired_o).astype(np.int32))
    stats_g = sim.read_counters(0, n_steps)
    if mode == ROUTE_TWO_LEVEL:
        stats_o[:, 5] = 0          # flat entries are only counted when flat routing runs
    if mode == ROUTE_FLAT:
        stats_o[:, 3:5] = 0
        stats_o[:, 6] = 0
    assert np.array_equal(stats_g, stats_o)
    g, o = _same_state(sim, orc, "end")
    # FP64 trajectory: device u within fp64_bound while the rasters agree
    acc = orc.accuracy()
    if fp64_bound is None:
        print(f"[gpu] {wl.name}: max |u - u_fp64| = {acc['max_dv']:.3e} mV, "
              f"max |u| = {np.max(np.abs(o['u64'])):.1f} mV", flush=True)
    else:
        if acc["first_divergence"] < 0:
            assert np.max(np.abs(g["u"].astype(np.float64) - o["u64"])) < fp64_bound
        assert acc["max_dv"] < fp64_bound
    return sim, orc, stats_o


@pytest.mark.parametrize("seed", [1, 2, 3])
@pytest.mark.parametrize("name", ["tiny", "tiny_active"])
def test_tiny_lockstep_1000_steps(name, seed):
    wl = synth.get_workload(name).replace(seed=seed)
    _, _, stats = _lockstep(wl, 1000, route_every=25, state_every=100)
    spikes = int(stats[:, 0].sum())
    print(f"[gpu] {name} seed {seed}: {spikes} spikes", flush=True)
    assert spikes > (10_000 if name == "tiny_active" else 100)


@pytest.mark.parametrize("mode", [ROUTE_TWO_LEVEL, ROUTE_BOTH, ROUTE_FLAT])
@pytest.mark.parametrize("name", ["tiny", "tiny_active"])
def test_fused_route_lockstep(name, mode):
    """snn_step_route (two-level routing inside the update kernel; flat mode
    takes the separate kernels) against the oracle: the same buckets, lists,
    counters and state."""
    wl = synth.get_workload(name).replace(seed=4)
    _lockstep(wl, 300, route_every=10, state_every=50, mode=mode, fused=True)


def test_connection_counts_match_oracle():
    """Per-list sizes without the entries (snn_read_routes with entries = NULL,
    as the bench reads the connections of a step): partitions and nodes
    reached and the message counts per node equal the oracle's."""
    wl = synth.get_workload("tiny_active").replace(seed=5)
    sim, orc = _pair(wl, log_steps=50)
    for _ in range(50):
        sim.step_route(ROUTE_TWO_LEVEL)
        sim.deliver()
        orc.step()
        per_part = sim.route_sizes(1)
        per_node = sim.route_sizes(2)
        assert np.array_equal(per_part, np.array([len(x) for x in orc.recv(1)], np.uint64))
        assert np.array_equal(per_node, np.array([len(x) for x in orc.buckets()], np.uint64))


@pytest.mark.parametrize("name", ["tiny_active", "batched"])
def test_link_traffic_matches_fired_sources(name):
    """Per-link traffic from the device buffers (links.link_traffic) against the
    same matrices built directly from the oracle's fired neurons and the
    destination lists: entries per (source partition, destination partition),
    messages per (source partition, destination node), level 1 / level 2."""
    from paper_2205_07125_amd.links import link_traffic
    wl = synth.get_workload(name)
    if name == "batched":
        wl = wl.scaled(12_000)
    sim, orc = _pair(wl, log_steps=30)
    host = sim.host
    P, G = wl.n_partitions, wl.gpus_per_node
    for t in range(30):
        sim.step_route(ROUTE_TWO_LEVEL)
        sim.deliver()
        orc.step()
        if t % 10 != 9:
            continue
        got = link_traffic(sim, host.part)
        pm = np.zeros((P, P), np.int64)
        nm = np.zeros((P, wl.n_nodes), np.int64)
        for s in orc.fired():
            dst = host.vp_part[host.vp_ptr[s]:host.vp_ptr[s + 1]].astype(np.int64)
            pm[host.part[s], dst] += 1
            nm[host.part[s], np.unique(dst // G)] += 1
        assert np.array_equal(got["partition_matrix"], pm)
        assert np.array_equal(got["node_matrix"], nm)
        own = nm[np.arange(P), np.arange(P) // G].sum()
        assert got["level1"] == own and got["level2"] == nm.sum() - own
        st = sim.read_counters(t, 1)[0]
        assert got["level1"] == st[3] and got["level2"] == st[4]     # msg_l1, msg_l2


def test_fused_route_many_spikes_per_tile():
    """60 % of one tile firing per step (the whole network as one 8,192-neuron
    tile): more fired neurons than a routing batch holds (512) and more pairs
    than a window holds (1,728 at this node count), so the batch and window
    loops of the fused routing
    run, with runs of one node cut by a window's end; each node gets more
    messages than one expansion round loads (2,048) and more entries than the
    staging buffer holds (4,096)."""
    wl = synth.get_workload("tiny").replace(name="tiny_dense", forced=1, rate_on_hz=6000.0,
                                            rate_off_hz=6000.0, period_steps=1, on_steps=1)
    _, _, stats = _lockstep(wl, 30, route_every=1, state_every=10, mode=ROUTE_BOTH, fused=True,
                            tile_neurons=8192)
    assert stats[:, 0].min() > 2048
    assert stats[:, 6].min() > 2 * 2 * 4096    # two nodes, each over two buffers


@pytest.mark.parametrize("tile", [64, 320, 1216, 8192])
def test_tile_sizes_match_oracle(tile):
    """Tiles of 64 neurons (64 tiles), of sizes that are no power of two and
    leave a partial last tile (320: 13 tiles, the last of 256 neurons; 1,216:
    4 tiles, the last of 448), and the whole network in one tile: the update's
    partial quads, the division of target ids by the tile size in the delivery,
    and the look-back over many tiles, in both step forms."""
    wl = synth.get_workload("tiny_active")
    _lockstep(wl, 40, route_every=7, state_every=20, mode=ROUTE_BOTH, tile_neurons=tile)
    _lockstep(wl, 40, route_every=7, state_every=20, mode=ROUTE_TWO_LEVEL, fused=True,
              tile_neurons=tile)


def test_unfused_fallback_many_nodes():
    """2,000 nodes of one GPU: more than the fused routing's LDS counters hold,
    so snn_step_route falls back to the routing kernel."""
    wl = synth.get_workload("paper_share").scaled(20_000, gpus_per_node=1)
    _lockstep(wl, 40, route_every=5, state_every=20, mode=ROUTE_TWO_LEVEL, fused=True)


def test_direct_route_beyond_lds_nodes():
    """5,000 nodes of one GPU: more than the routing kernel's LDS counters
    hold (4,096), so two-level routing takes the unstaged kernel (one atomic
    per message); buckets, lists and state against the oracle."""
    wl = synth.get_workload("paper_share").scaled(20_000, n_partitions=5000, gpus_per_node=1)
    assert wl.n_nodes > 4096
    _lockstep(wl, 30, route_every=5, state_every=15, mode=ROUTE_BOTH)


def test_route_modes_give_identical_rasters():
    wl = synth.get_workload("tiny_active")
    from paper_2205_07125_amd import Simulation
    a = Simulation(wl, log_steps=400)
    b = Simulation(wl, log_steps=400)
    for _ in range(400):
        a.full_step(ROUTE_TWO_LEVEL)
        b.full_step(ROUTE_FLAT)
    ia, ca = a.read_spikes(0, 400)
    ib, cb = b.read_spikes(0, 400)
    assert np.array_equal(ia, ib) and np.array_equal(ca, cb)
    sa, sb = a.state(), b.state()
    for k in ("u", "ref", "ring"):
        assert np.array_equal(sa[k], sb[k])
    ka, kb = a.read_counters(0, 400), b.read_counters(0, 400)
    # same deliveries; two-level sends fewer messages than flat
    assert np.array_equal(ka[:, :3], kb[:, :3])
    assert np.array_equal(ka[:, 6], kb[:, 5])           # expanded entries = flat entries
    assert np.all(ka[:, 3] + ka[:, 4] <= kb[:, 5])


def _oracle_steps(orc, n):
    """n oracle steps -> (fired ids of each step, counters in device order)."""
    fired, stats = [], np.zeros((n, 7), np.uint64)
    for t in range(n):
        orc.step()
        fired.append(orc.fired())
        stats[t] = orc.counters()[STAT_MAP]
    return fired, stats


def test_graph_replay_matches_oracle():
    """snn_run replaying captured steps (16-step graphs, then one-step graphs
    for the remainder) in both route modes equals the oracle: fired ids of
    every step, all seven counters, and the state."""
    wl = synth.get_workload("tiny_active").replace(seed=7)
    n = [150, 150, 17]               # 9 x 16 + 6 x 1, again in flat mode, then 16 + 1
    modes = [ROUTE_TWO_LEVEL, ROUTE_FLAT, ROUTE_TWO_LEVEL]
    sim, orc = _pair(wl, log_steps=sum(n))
    fired, stats = [], []
    for k, mode in zip(n, modes):
        sim.run(k, mode, use_graph=True)
        f, st = _oracle_steps(orc, k)
        if mode == ROUTE_TWO_LEVEL:
            st[:, 5] = 0              # flat entries are counted only when flat routing runs
        else:
            st[:, 3:5] = 0
            st[:, 6] = 0
        fired += f
        stats.append(st)
        _same_state(sim, orc, f"after {len(fired)} graph steps")
    ids, counts = sim.read_spikes(0, len(fired))
    assert np.array_equal(counts, np.array([len(f) for f in fired], np.uint32))
    assert np.array_equal(ids, np.concatenate(fired).astype(np.int32))
    assert np.array_equal(sim.read_counters(0, len(fired)), np.concatenate(stats))


def test_graph_and_eager_agree():
    wl = synth.get_workload("tiny_active").replace(seed=9)
    from paper_2205_07125_amd import Simulation
    a = Simulation(wl, log_steps=200)
    b = Simulation(wl, log_steps=200)
    a.run(200, ROUTE_TWO_LEVEL, use_graph=True)
    b.run(200, ROUTE_TWO_LEVEL, use_graph=False)
    sa, sb = a.state(), b.state()
    for k in ("u", "ref", "ring"):
        assert np.array_equal(sa[k], sb[k])


def test_bf16_weights_identical_for_dyadic():
    wl = synth.get_workload("tiny_active")
    from paper_2205_07125_amd import Simulation
    a = Simulation(wl, log_steps=300)
    b = Simulation(wl.replace(weight_type="bf16"), log_steps=300)
    a.run(300, ROUTE_TWO_LEVEL, use_graph=False)
    b.run(300, ROUTE_TWO_LEVEL, use_graph=False)
    sa, sb = a.state(), b.state()
    for k in ("u", "ref", "ring"):
        assert np.array_equal(sa[k], sb[k])


def test_forced_raster_matches_oracle():
    wl = synth.get_workload("heavy").scaled(3000, k_in=300, vp_set_size=40, period_steps=50,
                                            on_steps=10)
    _lockstep(wl, 120, route_every=10, state_every=40)
