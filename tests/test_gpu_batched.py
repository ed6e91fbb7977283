"""Many uneven partitions on one GPU: the layouts and launch shapes that the
batched form chooses between give identical results.

* one update launch over all partitions (tiles of neurons cross partition
  boundaries) against one update launch per partition (snn_run_partitioned);
* persistent update blocks (fewer blocks than tiles, tiles taken in turn)
  against one block per tile;
* the receive side with several blocks sharing one destination node's
  messages against one block per node, and as one launch against two;
* one HIP graph of all steps against 16-step graphs and eager launches;

and the per-partition layout against the oracle.  Routing buffers are
compared as multisets (their order is unspecified); everything else bit for
bit."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import STAT_MAP

pytestmark = pytest.mark.gpu

TWO_LEVEL = 0


def _wl(name):
    if name == "batched":
        return synth.get_workload("batched").scaled(58_000)    # 64 uneven partitions, 8 tiles
    if name == "paper_share":
        return synth.get_workload("paper_share").scaled(50_000)
    return synth.get_workload(name)


def _sims(wl, n, **kw):
    from paper_2205_07125_amd import HostNetwork, Simulation
    print(f"[gpu] {wl.name}: N={wl.n_neurons} P={wl.n_partitions} {kw}", flush=True)
    host = HostNetwork(wl)
    return Simulation(wl, host=host, log_steps=n), Simulation(wl, host=host, log_steps=n)


def _same(a, b, wl, n, where):
    ia, ca = a.read_spikes(0, n)
    ib, cb = b.read_spikes(0, n)
    assert ca.sum() > 0, where
    assert np.array_equal(ca, cb) and np.array_equal(ia, ib), f"fired ids, {where}"
    assert np.array_equal(a.read_counters(0, n), b.read_counters(0, n)), f"counters, {where}"
    ra, rb = a.read_routes(1), b.read_routes(1)
    for p in range(wl.n_partitions):
        assert np.array_equal(np.sort(ra[p]), np.sort(rb[p])), f"list {p}, {where}"
    sa, sb = a.state(), b.state()
    for k in ("u", "ref", "ring"):
        assert np.array_equal(sa[k].view(np.uint8), sb[k].view(np.uint8)), f"{k}, {where}"


@pytest.mark.parametrize("name", ["tiny_active", "batched", "paper_share"])
def test_partitioned_update_matches_one_launch(name):
    wl = _wl(name)
    n = 60
    a, b = _sims(wl, n + 32)
    a.run(n, TWO_LEVEL, use_graph=False)
    b.run_partitioned(n, TWO_LEVEL, use_graph=False)
    _same(a, b, wl, n, "eager")
    a.run(32, TWO_LEVEL, use_graph=True)
    b.run_partitioned(32, TWO_LEVEL, use_graph=True)
    _same(a, b, wl, n + 32, "graphs")


def test_partitioned_update_matches_oracle():
    """The per-partition layout of the 64 uneven partitions, step by step:
    fired ids and all seven counters of every step, the state at the end."""
    from paper_2205_07125_amd import HostNetwork, Simulation
    wl = _wl("batched")
    n = 40
    sim = Simulation(wl, host=HostNetwork(wl), log_steps=n)
    orc = oracle.sim_for_workload(wl)
    fired, stats = [], np.zeros((n, 7), np.uint64)
    for t in range(n):
        sim.run_partitioned(1, TWO_LEVEL, use_graph=False)
        orc.step()
        fired.append(orc.fired())
        stats[t] = orc.counters()[STAT_MAP]
    stats[:, 5] = 0                     # flat entries are counted only when flat routing runs
    ids, counts = sim.read_spikes(0, n)
    assert np.array_equal(counts, np.array([len(f) for f in fired], np.uint32))
    assert np.array_equal(ids, np.concatenate(fired).astype(np.int32))
    assert np.array_equal(sim.read_counters(0, n), stats)
    g, o = sim.state(), orc.state()
    assert np.array_equal(g["u"].view(np.uint32), o["u"].view(np.uint32))
    assert np.array_equal(g["ref"], o["ref"])
    assert np.array_equal(g["ring"].view(np.uint32), o["ring"].view(np.uint32))


@pytest.mark.parametrize("blocks", [1, 3, 5])
def test_persistent_update_matches(blocks):
    wl = _wl("batched")
    n = 50
    a, b = _sims(wl, n, update_blocks=blocks)
    b.set_tuning(update_blocks=blocks)
    assert b.tuning()["update_blocks"] == blocks
    a.run(n, TWO_LEVEL, use_graph=False)
    b.run(n, TWO_LEVEL, use_graph=False)
    _same(a, b, wl, n, f"{blocks} persistent blocks")


@pytest.mark.parametrize("split", [1, 2, 7])
@pytest.mark.parametrize("name", ["tiny_active", "batched"])
def test_recv_split_matches(name, split):
    wl = _wl(name)
    n = 50
    a, b = _sims(wl, n, recv_split=split)
    b.set_tuning(recv_split=split)
    a.run(n, TWO_LEVEL, use_graph=False)
    b.run(n, TWO_LEVEL, use_graph=False)
    _same(a, b, wl, n, f"recv_split {split}")


@pytest.mark.parametrize("name", ["tiny_active", "batched", "paper_share"])
def test_recv_merged_matches(name):
    """The receive side as one launch (delivery blocks wait for the staging
    blocks on their XCD and read their queues through its L2; the default)
    against two launches."""
    wl = _wl(name)
    n = 60
    a, b = _sims(wl, n, recv_merged=1)
    a.set_tuning(recv_merged=0)
    b.set_tuning(recv_merged=1)
    assert a.tuning()["recv_merged"] == 0 and b.tuning()["recv_merged"] == 1
    a.run(n, TWO_LEVEL, use_graph=False)
    b.run(n, TWO_LEVEL, use_graph=True)
    _same(a, b, wl, n, "one receive launch")


def test_recv_merged_matches_oracle():
    """One receive launch, step by step against the oracle (64 uneven
    partitions, several blocks per destination node)."""
    from paper_2205_07125_amd import HostNetwork, Simulation
    wl = _wl("batched")
    n = 40
    sim = Simulation(wl, host=HostNetwork(wl), log_steps=n)
    sim.set_tuning(recv_merged=1)
    orc = oracle.sim_for_workload(wl)
    fired, stats = [], np.zeros((n, 7), np.uint64)
    for t in range(n):
        sim.run(1, TWO_LEVEL, use_graph=False)
        orc.step()
        fired.append(orc.fired())
        stats[t] = orc.counters()[STAT_MAP]
    stats[:, 5] = 0
    ids, counts = sim.read_spikes(0, n)
    assert np.array_equal(ids, np.concatenate(fired).astype(np.int32))
    assert np.array_equal(sim.read_counters(0, n), stats)
    g, o = sim.state(), orc.state()
    assert np.array_equal(g["u"].view(np.uint32), o["u"].view(np.uint32))
    assert np.array_equal(g["ring"].view(np.uint32), o["ring"].view(np.uint32))


def test_whole_run_graph():
    """use_graph = 2: one graph of all steps, captured, replayed again from the
    cache, and captured anew for another step count."""
    wl = _wl("tiny_active")
    a, b = _sims(wl, 230)
    for k in (100, 100, 30):
        a.run(k, TWO_LEVEL, use_graph=2)
        b.run(k, TWO_LEVEL, use_graph=False)
    _same(a, b, wl, 230, "whole-run graph")
