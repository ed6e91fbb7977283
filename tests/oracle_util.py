"""Helpers to build small hand-made networks for the oracle's pin tests."""
import numpy as np

import oracle


def make_sim(n, edges=None, part=None, u0=None, **over):
    """A network of n neurons with explicit synapses
    edges = [(src, tgt, delay, vp, w), ...]."""
    edges = edges or []
    arr = dict(
        src=np.array([e[0] for e in edges], np.uint32),
        tgt=np.array([e[1] for e in edges], np.uint32),
        delay=np.array([e[2] for e in edges], np.uint8),
        vp=np.array([e[3] for e in edges], np.uint16),
        w=np.array([e[4] for e in edges], np.float32),
    )
    kw = dict(n_neurons=n, n_partitions=1, gpus_per_node=1, max_delay=10, dt_ms=0.1,
              tau_m_ms=20.0, theta_mv=15.0, u_reset_mv=0.0, t_ref_ms=2.0, nu_ext_hz=0.0,
              w_ext_mv=0.0, seed=3, forced=0, period_steps=1, on_steps=0, rate_on_hz=0.0,
              rate_off_hz=0.0, bf16_weights=0)
    kw.update(over)
    params = oracle.Params(**kw)
    if part is None:
        part = np.zeros(n, np.int32)
    if u0 is None:
        u0 = np.zeros(n, np.float32)
    return oracle.Sim(params, arr, np.asarray(part, np.int32), np.asarray(u0, np.float32))
