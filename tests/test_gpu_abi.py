"""C ABI behaviour on the device: phase order, sticky capacity overflow
(forced with tiny bounds; nothing is truncated silently), spike-log limits,
read-back preconditions, determinism of repeated runs."""
import numpy as np
import pytest

import synth
from paper_2205_07125_amd import Simulation, _abi

pytestmark = pytest.mark.gpu


def _wl():
    return synth.get_workload("tiny_active")


def test_phase_order_enforced():
    sim = Simulation(_wl(), log_steps=10)
    with pytest.raises(_abi.SNNError) as e:
        sim.route(0)
    assert e.value.status == _abi.SNN_ERR_BAD_STATE
    with pytest.raises(_abi.SNNError):
        sim.deliver()
    with pytest.raises(_abi.SNNError):
        sim.read_routes(1)            # nothing routed yet
    sim.step()
    with pytest.raises(_abi.SNNError) as e:
        sim.step()
    assert e.value.status == _abi.SNN_ERR_BAD_STATE
    with pytest.raises(_abi.SNNError):
        sim.run(3, 0)                 # in the middle of a step
    sim.route(1)
    with pytest.raises(_abi.SNNError):
        sim.read_routes(1)            # flat mode filled only the flat lists
    sim.deliver()
    assert sim.t == 1
    sim.read_routes(0)
    with pytest.raises(_abi.SNNError):
        sim.route(7)


@pytest.mark.parametrize("which", ["bucket", "recv"])
def test_capacity_overflow_is_reported(which):
    wl = _wl()
    from paper_2205_07125_amd import HostNetwork
    host = HostNetwork(wl)
    kw = {}
    if which == "bucket":
        kw["bucket_off"] = np.arange(wl.n_nodes + 1, dtype=np.uint64)        # 1 per node
    else:
        kw["recv_off"] = np.arange(wl.n_partitions + 1, dtype=np.uint64)     # 1 per partition
    sim = Simulation(wl, host=host, log_steps=20, **kw)
    sim.run(20, _abi.SNN_ROUTE_BOTH, use_graph=False)
    with pytest.raises(_abi.SNNError) as e:
        sim.sync()
    assert e.value.status == _abi.SNN_ERR_CAPACITY
    # sticky: still reported later
    with pytest.raises(_abi.SNNError):
        sim.read_routes(1)


def test_spike_log_limits():
    sim = Simulation(_wl(), log_steps=5, log_cap=4)
    sim.run(30, 0, use_graph=False)
    with pytest.raises(_abi.SNNError) as e:
        sim.read_spikes(0, 5)         # older than the last 5 steps
    assert e.value.status == _abi.SNN_ERR_INVALID_ARG
    with pytest.raises(_abi.SNNError) as e:
        sim.sync()                    # some step had more than 4 spikes
    assert e.value.status == _abi.SNN_ERR_CAPACITY


def test_repeated_runs_bit_identical():
    wl = synth.get_workload("paper_share").scaled(40_000)
    a = Simulation(wl, log_steps=60)
    b = Simulation(wl, log_steps=60)
    a.run(60, 0, use_graph=True)
    b.run(60, 0, use_graph=True)
    sa, sb = a.state(), b.state()
    for k in ("u", "ref", "ring"):
        assert np.array_equal(sa[k].view(np.uint8), sb[k].view(np.uint8))
    assert np.array_equal(a.read_counters(0, 60), b.read_counters(0, 60))
    ia, _ = a.read_spikes(0, 60)
    ib, _ = b.read_spikes(0, 60)
    assert np.array_equal(ia, ib)


def test_empty_steps():
    """A silent network (no drive, no initial suprathreshold neurons) routes
    and delivers nothing, and every counter stays zero."""
    wl = _wl().replace(w_ext_mv=0.0, name="silent")
    sim = Simulation(wl, log_steps=20)
    sim.u.zero_()
    import torch
    torch.cuda.synchronize()
    sim.run(20, _abi.SNN_ROUTE_BOTH, use_graph=False)
    assert np.all(sim.read_counters(0, 20) == 0)
    ids, counts = sim.read_spikes(0, 20)
    assert len(ids) == 0 and np.all(counts == 0)
    assert all(len(x) == 0 for x in sim.read_routes(1))


@pytest.mark.parametrize("jitter", [0.0, 0.2])
@pytest.mark.parametrize("bin_cap,stage_cap", [(0, 0), (2, 1)])
def test_dense_ring_fallback_is_exact(bin_cap, stage_cap, jitter):
    """With no (or tiny) bin and staging capacity every event takes the dense
    overflow path; the result is the same as with the bins, bit for bit, also
    with non-dyadic (jittered) weights: both paths sum the same fixed-point
    weights exactly."""
    wl = synth.get_workload("tiny_active").replace(w_jitter=jitter)
    a = Simulation(wl, log_steps=150)
    b = Simulation(wl, log_steps=150, bin_cap=bin_cap, stage_cap=stage_cap)
    a.run(150, _abi.SNN_ROUTE_TWO_LEVEL, use_graph=False)
    b.run(150, _abi.SNN_ROUTE_TWO_LEVEL, use_graph=False)
    assert b.ring_events() > 0
    sa, sb = a.state(), b.state()
    for k in ("u", "ref", "ring"):
        assert np.array_equal(sa[k], sb[k]), k
    ia, _ = a.read_spikes(0, 150)
    ib, _ = b.read_spikes(0, 150)
    assert np.array_equal(ia, ib)


def test_state_reads_leave_the_run_unchanged():
    """Reading the state (snn_flush) between steps only reads: with jittered
    (non-dyadic) weights a run read every 7 steps equals one never read."""
    wl = synth.get_workload("tiny_active").replace(w_jitter=0.2)
    a = Simulation(wl, log_steps=120)
    b = Simulation(wl, log_steps=120)
    for t in range(120):
        a.full_step(_abi.SNN_ROUTE_TWO_LEVEL)
        b.full_step(_abi.SNN_ROUTE_TWO_LEVEL)
        if t % 7 == 3:
            a.state()
    ia, ca = a.read_spikes(0, 120)
    ib, cb = b.read_spikes(0, 120)
    assert ca.sum() > 0 and np.array_equal(ca, cb) and np.array_equal(ia, ib)
    sa, sb = a.state(), b.state()
    for k in ("u", "ref", "ring"):
        assert np.array_equal(sa[k].view(np.uint8), sb[k].view(np.uint8)), k
