"""Pins of the oracle's synaptic delivery: the ring increment equals the dense
FP64 product W_d^T 1_F (numpy), event counts equal out-degree sums, ring mass
is conserved.  CPU only."""
import numpy as np
import pytest

import oracle
from oracle_util import make_sim


def _dense(n, edges, D):
    W = np.zeros((D, n, n), np.float64)   # W[d, src, tgt], repeated pairs summed
    for s, t, d, _, w in edges:
        W[d, s, t] += w
    return W


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_ring_increment_is_dense_product(seed):
    rng = np.random.default_rng(seed)
    n, m, P = 40, 600, 4
    part = (np.arange(n) * P // n).astype(np.int32)
    src = rng.integers(0, n, m)
    tgt = rng.integers(0, n, m)
    keep = src != tgt
    edges = [(int(s), int(t), int(rng.integers(1, 11)), int(part[t]),
              0.5 if s % 5 != 4 else -2.5) for s, t in zip(src[keep], tgt[keep])]
    u0 = np.where(rng.random(n) < 0.3, 20.0, 0.0).astype(np.float32)
    sim = make_sim(n, edges=edges, part=part, u0=u0, n_partitions=P, gpus_per_node=2)
    sim.step()
    fired = sim.fired()
    ind = np.zeros(n)
    ind[fired] = 1.0
    W = _dense(n, edges, 11)
    st = sim.state()
    for d in range(1, 11):
        want = W[d].T @ ind            # slot (0 + d) mod 11
        assert np.array_equal(st["ring64"][d], want)
        assert np.array_equal(st["ring"][d].astype(np.float64), want)   # dyadic: exact
    assert np.all(st["ring"][0] == 0)  # slot of step 0 was consumed and cleared
    # I3: delivered events = sum of out-degrees of fired sources
    outdeg = np.bincount([e[0] for e in edges], minlength=n)
    c = sim.counters()
    assert c[oracle.LOCAL_EVENTS] + c[oracle.REMOTE_EVENTS] == outdeg[fired].sum()
    local = sum(1 for e in edges if ind[e[0]] and part[e[0]] == e[3])
    assert c[oracle.LOCAL_EVENTS] == local
    # I7: ring mass = sum of delivered weights
    assert st["ring64"].sum() == sum(e[4] for e in edges if ind[e[0]])


def test_whole_step_invariants_tiny():
    """I8 on the tiny active net: fired neurons sit at reset with a full
    refractory count, integrating non-fired neurons are below threshold."""
    import synth
    wl = synth.get_workload("tiny_active")
    sim = oracle.sim_for_workload(wl)
    for t in range(80):
        sim.step()
        st = sim.state()
        f = sim.fired()
        assert np.all(st["u"][f] == 0.0) and np.all(st["ref"][f] == 20)
        mask = np.ones(wl.n_neurons, bool)
        mask[f] = False
        assert np.all(st["u"][mask & (st["ref"] == 0)] < 15.0)


def test_bf16_weights_dyadic_identical():
    """BF16 rounding is lossless on the stated dyadic weights: the BF16 run is
    bit-identical to the FP32 run."""
    import synth
    wl = synth.get_workload("tiny_active")
    a = oracle.sim_for_workload(wl)
    b = oracle.sim_for_workload(wl.replace(weight_type="bf16"))
    for _ in range(100):
        assert a.step() == b.step()
        assert np.array_equal(a.fired(), b.fired())
    sa, sb = a.state(), b.state()
    assert np.array_equal(sa["u"], sb["u"]) and np.array_equal(sa["ring"], sb["ring"])
