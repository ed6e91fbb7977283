"""The device path on layouts planned by the paper's setup (Sec. IV): a
clustered network is mapped to GPUs by Algorithm 1 (or by contiguous id
ranges, or at random, for comparison), the GPUs are grouped by Algorithm 2
and renumbered so that each group is one node, and the resulting neuron ->
partition map is what the device and the oracle both build the network from.
Groups of 16 and 40 partitions exercise node masks wider than 8 bits (up to
64).  Parity with the oracle in lockstep, and the traffic each map causes,
read from the device's counters and routing buffers."""
import numpy as np
import pytest

import synth
from paper_2205_07125_amd import partition as pt
from test_gpu_parity import ROUTE_BOTH, ROUTE_TWO_LEVEL, _lockstep

pytestmark = pytest.mark.gpu


def _planned(n, P, G, kind="alg1"):
    wl = synth.get_workload("clustered").scaled(n, n_partitions=P, gpus_per_node=G,
                                                n_clusters=P)
    e = synth.Generator(wl).edges()
    Pm, W = pt.connectivity(e["src"], e["tgt"], wl.n_neurons)
    pm, info = pt.device_map(Pm, W, P, G, kind, iters=2, seed=1)
    # groups are consecutive nodes of G partitions
    assert np.array_equal(info["new_id"] // G, info["group_of"])
    return wl, pm, e


@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
@pytest.mark.parametrize("G,P,n", [(16, 32, 16384), (40, 80, 20480), (64, 128, 16384)])
def test_planned_layout_lockstep(G, P, n, fused):
    """Algorithm 1's map and Algorithm 2's groups on the device: spikes,
    buckets (64-bit masks), receive lists, counters and state against the
    oracle on the same map."""
    wl, pm, _ = _planned(n, P, G)
    print(f"[gpu] planned layout G={G} P={P} N={n} fused={fused}", flush=True)
    _, _, stats = _lockstep(wl, 40, route_every=5, state_every=20, mode=ROUTE_BOTH, fused=fused,
                            part_map=pm)
    assert stats[:, 0].sum() > 0 and stats[:, 4].sum() > 0


def test_planned_map_cuts_remote_traffic():
    """The same clustered network under three maps, 60 steps each on the
    device: Algorithm 1's map keeps most synapses inside their partition, so
    far fewer events travel through receive lists and fewer entries and
    messages leave each partition than under contiguous or random maps."""
    from paper_2205_07125_amd import HostNetwork, Simulation
    from paper_2205_07125_amd.links import link_traffic
    rows = {}
    for kind in ("alg1", "contiguous", "random"):
        wl, pm, _ = _planned(16384, 32, 16, kind)
        host = HostNetwork(wl, part_map=pm)
        sim = Simulation(wl, host=host, log_steps=60)
        sim.run(59, ROUTE_TWO_LEVEL, use_graph=False)
        sim.step_route(ROUTE_TWO_LEVEL)
        sim.deliver()
        c = sim.read_counters(0, 60).astype(np.float64).sum(axis=0)
        lt = link_traffic(sim, host.part)
        rows[kind] = dict(remote_frac=c[2] / (c[1] + c[2]), entries_per_spike=c[6] / c[0],
                          msgs_per_spike=(c[3] + c[4]) / c[0],
                          peak_partition_entries=int(lt["partition_matrix"].sum(axis=1).max()),
                          peak_link=lt["max_partition_link"])
        print(f"[gpu] map {kind}: {rows[kind]}", flush=True)
        sim.close()
    a, c, r = rows["alg1"], rows["contiguous"], rows["random"]
    assert a["remote_frac"] < 0.6 * min(c["remote_frac"], r["remote_frac"])
    assert a["entries_per_spike"] < min(c["entries_per_spike"], r["entries_per_spike"])
    assert a["peak_partition_entries"] < min(c["peak_partition_entries"],
                                             r["peak_partition_entries"])
