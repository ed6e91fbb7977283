"""The GPU path's host setup (libsnn's snn_setup_* entry points) against the
seeded generator's synapse list, and its derived constants against the
oracle's.  CPU only: no kernel runs here."""
import numpy as np
import pytest

import oracle
import synth
from paper_2205_07125_amd import HostNetwork, derived_params


def _check_network(wl, host, part_map=None):
    """Vectorised comparison of the CSR layout with the canonical list."""
    gen = synth.Generator(wl, part_map=part_map)
    e = gen.edges()
    part = gen.part_map().astype(np.int64)
    N, G, P = wl.n_neurons, wl.gpus_per_node, wl.n_partitions
    assert np.array_equal(host.part, part)
    row_ptr = host.row_ptr
    row_len = np.diff(row_ptr)
    assert np.array_equal(row_len, np.bincount(e["src"], minlength=N))
    nnz = int(row_ptr[-1])
    src_h = np.repeat(np.arange(N), row_len)
    pos = np.arange(nnz) - row_ptr[src_h]
    nl = host.n_local.astype(np.int64)
    local = pos < nl[src_h]
    # destination-partition lists: distinct, ascending, never the own partition
    vp_ptr = host.vp_ptr
    n_vp = np.diff(vp_ptr)
    pairs = int(vp_ptr[-1])
    assert host.pairs == pairs
    vp_part = host.vp_part[:pairs].astype(np.int64)
    rec = host.vp_rec[:2 * pairs].reshape(-1, 2) if pairs else np.zeros((0, 2), np.uint64)
    seg_start = (rec[:, 0] & np.uint64((1 << 40) - 1)).astype(np.int64)
    seg_len = (rec[:, 0] >> np.uint64(40)).astype(np.int64)
    owner = np.repeat(np.arange(N), n_vp)
    first = np.zeros(pairs, bool)
    first[vp_ptr[:-1][n_vp > 0]] = True
    assert np.all(vp_part != part[owner])
    assert np.all(np.diff(vp_part)[~first[1:]] > 0)          # ascending within a source
    # segments: right after the local part, contiguous, ending at the row's end
    assert np.all(seg_start[first] == row_ptr[owner[first]] + nl[owner[first]])
    assert np.all(seg_start[1:][~first[1:]] == (seg_start + seg_len)[:-1][~first[1:]])
    last = np.append(first[1:], True)
    assert np.all((seg_start + seg_len)[last] == row_ptr[owner[last] + 1])
    assert np.all(seg_len > 0)
    assert seg_len.sum() == (~local).sum()
    # the record's copy of the segment's first synapse
    if pairs:
        assert np.array_equal((rec[:, 1] & np.uint64(0xFFFFFFFF)).astype(np.uint32),
                              host.tgt_delay[seg_start])
        wbits = (rec[:, 1] >> np.uint64(32)).astype(np.uint32)
        if wl.weight_type == "bf16":
            assert np.array_equal(wbits, host.weight[seg_start].astype(np.uint32))
        else:
            assert np.array_equal(wbits, host.weight.view(np.uint32)[seg_start])
    vp_h = np.empty(nnz, np.int64)
    vp_h[local] = part[src_h[local]]
    vp_h[~local] = np.repeat(vp_part, seg_len)
    # same multiset of synapses as the generator
    tgt_h = (host.tgt_delay & 0x07FFFFFF).astype(np.int64)
    d_h = (host.tgt_delay >> 27).astype(np.int64)
    if wl.weight_type == "bf16":
        import torch
        w_h = host.weight.astype(np.uint32) << 16
        w_g = torch.from_numpy(e["w"]).to(torch.bfloat16).to(torch.float32).numpy().view(np.uint32)
    else:
        w_h = host.weight.view(np.uint32)
        w_g = e["w"].view(np.uint32)
    a = np.stack([src_h, vp_h, tgt_h, d_h, w_h.astype(np.int64)])
    b = np.stack([e["src"], e["vp"], e["tgt"], e["delay"], w_g]).astype(np.int64)
    a = a[:, np.lexsort(a[::-1])]
    b = b[:, np.lexsort(b[::-1])]
    assert np.array_equal(a, b)
    # local segment = exactly the synapses whose destination is the own partition
    assert np.array_equal(local, vp_h == part[src_h])
    # input bound: the largest sum of |w| (as stored) over a neuron's inputs,
    # rounded up to a float
    w_abs = np.abs(w_g.view(np.float32).astype(np.float64))
    want = np.bincount(e["tgt"], weights=w_abs, minlength=N).max()
    assert np.float32(host.input_bound) >= want
    assert np.float32(host.input_bound) <= np.nextafter(np.float32(want), np.float32(np.inf))
    # exact capacity bounds: sources per destination partition / per node
    assert np.array_equal(np.diff(host.recv_off.astype(np.int64)), np.bincount(vp_part, minlength=P))
    node_pairs = np.unique(owner * (P // G + 1) + vp_part // G)
    assert np.array_equal(np.diff(host.bucket_off.astype(np.int64)),
                          np.bincount(node_pairs % (P // G + 1), minlength=wl.n_nodes))


@pytest.mark.parametrize("name", ["tiny", "tiny_bf16", "loopback_small", "sets_small",
                                  "batched_small"])
def test_setup_matches_generator(name):
    base = {
        "tiny": synth.get_workload("tiny"),
        "tiny_bf16": synth.get_workload("tiny").replace(weight_type="bf16", w_jitter=0.2),
        "loopback_small": synth.get_workload("paper_share").scaled(3000, k_in=60),
        "sets_small": synth.get_workload("heavy").scaled(1500, k_in=200, vp_set_size=30),
        "batched_small": synth.get_workload("batched").scaled(3000),
    }[name]
    host = HostNetwork(base, n_threads=4)
    _check_network(base, host)


def _clustered_small():
    return synth.get_workload("clustered").scaled(6000, k_in=40, n_partitions=12,
                                                  gpus_per_node=12, n_clusters=10)


def test_setup_clustered_with_partition_map():
    """An explicit neuron -> partition map (scattered, as a partitioning of
    the clustered net would give) is what the setup's rows, destination
    lists and own-partition segments follow; wide nodes (12 partitions)."""
    wl = _clustered_small()
    pm = np.random.default_rng(3).integers(0, wl.n_partitions, wl.n_neurons).astype(np.int32)
    host = HostNetwork(wl, n_threads=3, part_map=pm)
    assert np.array_equal(host.part, pm)
    _check_network(wl, host, part_map=pm)
    # the default contiguous ranges too
    _check_network(wl, HostNetwork(wl, n_threads=3))


def test_clustered_generator_statistics():
    """Clustered topology: no autapses, the fraction of inputs from the
    target's own cluster is p_in plus the chance share of the rest, and the
    clusters are scattered over the neuron ids."""
    wl = _clustered_small().replace(p_in=0.7)
    gen = synth.Generator(wl)
    e = gen.edges()
    cl = gen.clusters().astype(np.int64)
    assert np.all(e["src"] != e["tgt"])
    same = cl[e["src"]] == cl[e["tgt"]]
    share = np.bincount(cl, minlength=wl.n_clusters) / wl.n_neurons
    want = wl.p_in + (1 - wl.p_in) * float(np.sum(share ** 2))
    m = len(same)
    assert abs(same.mean() - want) < 5 * np.sqrt(want * (1 - want) / m)
    # scattered: a contiguous block of ids holds many clusters
    assert len(np.unique(cl[:500])) == wl.n_clusters
    with pytest.raises(ValueError):
        synth.Generator(wl, part_map=np.full(wl.n_neurons, wl.n_partitions, np.int32))
    with pytest.raises(ValueError):
        synth.Generator(synth.get_workload("paper_share").scaled(2000),
                        part_map=np.zeros(2000, np.int32))


def test_setup_independent_of_threads():
    wl = synth.get_workload("paper_share").scaled(4000, k_in=50)
    a = HostNetwork(wl, n_threads=1)
    b = HostNetwork(wl, n_threads=7)
    for k in ("row_ptr", "n_local", "tgt_delay", "weight", "vp_ptr", "vp_part", "vp_rec",
              "bucket_off", "recv_off"):
        assert np.array_equal(getattr(a, k), getattr(b, k)), k
    assert a.input_bound == b.input_bound


@pytest.mark.parametrize("name", ["tiny", "paper_share", "heavy"])
def test_derived_params_match_oracle(name):
    wl = synth.get_workload(name)
    dp = derived_params(wl)
    p = oracle.params_from_workload(wl)
    assert np.float32(dp["alpha"]) == oracle.alpha(p)
    assert list(dp["poisson_thr"]) == list(oracle.poisson_table(wl.nu_ext_hz * wl.dt_ms * 1e-3))
    assert dp["n_ref"] == oracle.n_ref(p)
    assert dp["raster_thr_on"] == oracle.raster_threshold(wl.rate_on_hz, wl.dt_ms)
    assert dp["raster_thr_off"] == oracle.raster_threshold(wl.rate_off_hz, wl.dt_ms)


def test_model_params_rejects_bad_constants():
    from paper_2205_07125_amd import _abi
    good = dict(dt_ms=0.1, tau_m_ms=20.0, theta_mv=20.0, u_reset_mv=10.0, t_ref_ms=2.0,
                nu_ext_hz=8000.0, w_ext_mv=0.1, rate_on_hz=5.0, rate_off_hz=5.0)
    p = _abi.snn_setup_model_params(_abi.snn_params(n_neurons=7), **good)
    assert p.n_neurons == 7 and p.n_ref == 20          # other fields untouched
    assert list(p.poisson_thr) == sorted(p.poisson_thr)
    for bad in (dict(dt_ms=0.0), dict(tau_m_ms=-1.0), dict(nu_ext_hz=-1.0),
                dict(rate_on_hz=-5.0), dict(t_ref_ms=26.0), dict(dt_ms=float("nan"))):
        with pytest.raises(_abi.SNNError) as e:
            _abi.snn_setup_model_params(_abi.snn_params(), **dict(good, **bad))
        assert e.value.status == _abi.SNN_ERR_INVALID_ARG
