"""Parity with the oracle on reduced-size versions of every workload (same
in-degree structure, partitions, node grouping, topology and drive), in
lockstep with the routing buffers compared every few steps."""
import numpy as np
import pytest

import oracle
import synth
from test_gpu_parity import ROUTE_BOTH, _lockstep

pytestmark = pytest.mark.gpu


SCALED = {
    # 1/100 of the 5e6-neuron share, full in-degree and 2,000 partitions
    "paper_share": lambda: synth.get_workload("paper_share").scaled(50_000),
    "paper_share_lif": lambda: synth.get_workload("paper_share_lif").scaled(20_000),
    "paper_share_4k": lambda: synth.get_workload("paper_share_4k").scaled(50_000),
    "paper_share_bf16": lambda: synth.get_workload("paper_share_bf16").scaled(30_000),
    # 64 uneven partitions at 1/100
    "batched": lambda: synth.get_workload("batched").scaled(58_000),
    # heavy traffic: 200 partitions per source, bursts; in-degree cut so the
    # oracle stays small
    "heavy": lambda: synth.get_workload("heavy").scaled(12_000, k_in=1500, period_steps=40,
                                                        on_steps=10),
    # the same at the full in-degree of 10,000 (1.2e8 synapses, bins sized
    # for bursts of 1.2e6 events per step)
    "heavy_full_k": lambda: synth.get_workload("heavy").scaled(12_000, period_steps=40,
                                                               on_steps=10),
}


# Where the absolute FP64 bound of 1e-4 mV does not apply, and what bounds the
# drift instead.  At the full in-degree of 10,000, inhibition drives |u| to
# about 400 mV, where binary32's spacing is 2^-15 mV (3e-5): the roundings of
# a step (u * alpha, k * w_ext, syn + ext, the sum) add at most 2 ulp(max|u|),
# and alpha < 1 shrinks what earlier steps left, so before any raster
# divergence |u32 - u64| <= 2 * steps * ulp(max|u|).  The device must still
# equal the oracle's binary32 trajectory bit for bit.
ULP_BOUND = {"heavy_full_k"}


def ulp32(x: float) -> float:
    """Spacing of binary32 values at magnitude x (normal range)."""
    return 2.0 ** (np.floor(np.log2(x)) - 23)


@pytest.mark.parametrize("fused", [False, True], ids=["separate", "fused"])
@pytest.mark.parametrize("name", sorted(SCALED))
def test_scaled_workload_lockstep(name, fused):
    """fused: snn_step_route + snn_deliver, as snn_run launches a step (routing
    inside the update; expansion, staging and local delivery in one launch);
    paper_share_4k's 500 nodes run the staging blocks' node loop and come
    close to the fused routing's node limit."""
    wl = SCALED[name]()
    steps = 80
    _, orc, stats = _lockstep(wl, steps, route_every=8, state_every=40, mode=ROUTE_BOTH,
                              fused=fused, fp64_bound=None if name in ULP_BOUND else 1e-4)
    assert stats[:, 0].sum() > 0
    if name in ULP_BOUND:
        acc = orc.accuracy()
        bound = 2 * steps * ulp32(acc["max_abs_u"])
        print(f"[gpu] {name}: max |u - u_fp64| = {acc['max_dv']:.3e} mV, max |u| = "
              f"{acc['max_abs_u']:.1f} mV, bound {bound:.3e}", flush=True)
        assert acc["first_divergence"] < 0 and acc["max_dv"] <= bound
    print(f"[gpu] {name}: {int(stats[:, 0].sum())} spikes, "
          f"{int(stats[:, 1].sum() + stats[:, 2].sum())} events, "
          f"{int(stats[:, 3].sum() + stats[:, 4].sum())} two-level msgs, "
          f"{int(stats[:, 5].sum())} flat", flush=True)
