"""Host setup of a workload's network through libsnn's setup entry points,
then upload to device memory (torch tensors, caller-owned by the
Simulation)."""
from __future__ import annotations

import ctypes
import sys
import time

import numpy as np

from . import _abi

_P = ctypes.c_void_p


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_P)


def default_caps(wl, host, tile_neurons: int = 0) -> tuple[int, int]:
    """Bin and staging capacities sized at four times the expected events per
    bin at the workload's highest rate (50 Hz assumed for LIF-driven spikes);
    events beyond them take the dense-ring path, so these set speed, not
    correctness."""
    rate = max(wl.rate_on_hz, wl.rate_off_hz) if wl.forced else 50.0
    spikes = wl.n_neurons * rate * wl.dt_ms * 1e-3
    outdeg = host.nnz / max(wl.n_neurons, 1)
    local = float(host.n_local.sum()) / max(wl.n_neurons, 1)
    e_local = spikes * local
    e_remote = spikes * (outdeg - local)
    md = wl.max_delay
    tile, deliver_blocks, stage_blocks = _abi.snn_bin_geometry(wl.n_neurons, tile_neurons)
    tiles = (wl.n_neurons + tile - 1) // tile
    per_bin = (e_local + e_remote) / (md * deliver_blocks * tiles)
    per_queue = e_remote / (md * stage_blocks)
    rnd = lambda x: int(-(-(4 * x + 64) // 32) * 32)
    return rnd(per_bin), rnd(per_queue)


def derived_params(wl) -> dict:
    """Constants the kernels take ready-made, computed by the library from
    the workload's physical ones (snn_setup_model_params): the per-step decay
    factor fl32(exp(-dt / tau_m)), the Poisson inversion table
    floor(2^32 CDF(j)) for lambda = nu_ext dt, the refractory length and the
    forced-raster thresholds floor(2^32 rate dt)."""
    p = _abi.snn_setup_model_params(
        _abi.snn_params(), dt_ms=wl.dt_ms, tau_m_ms=wl.tau_m_ms, theta_mv=wl.theta_rel_mv,
        u_reset_mv=wl.u_reset_mv, t_ref_ms=wl.t_ref_ms, nu_ext_hz=wl.nu_ext_hz,
        w_ext_mv=wl.w_ext_mv, rate_on_hz=wl.rate_on_hz, rate_off_hz=wl.rate_off_hz)
    return dict(alpha=float(p.alpha), theta=float(p.theta), u_reset=float(p.u_reset),
                w_ext=float(p.w_ext), n_ref=int(p.n_ref), poisson_thr=list(p.poisson_thr),
                raster_thr_on=int(p.raster_thr_on), raster_thr_off=int(p.raster_thr_off))


class HostNetwork:
    """Arrays of include/snn.h's snn_network_dev, built on the host.
    part_map: explicit neuron -> partition map (the neuron-GPU mapping PM of
    Sec. IV-A) in place of the workload's contiguous partitions."""

    def __init__(self, wl, n_threads: int = 0, verbose: bool = False,
                 part_map: np.ndarray | None = None):
        import synth  # seeded input description (partition starts, cross fractions)
        self.wl = wl
        L = _abi.lib()
        spec = _abi.snn_setup_spec(
            seed=wl.seed, n_neurons=wl.n_neurons, k_in=wl.k_in, max_delay=wl.max_delay,
            n_partitions=wl.n_partitions, topology=wl.topology, vp_set_size=wl.vp_set_size,
            remote_frac=wl.remote_frac, w_exc=wl.w_exc, w_inh=wl.w_inh, w_jitter=wl.w_jitter,
            gpus_per_node=wl.gpus_per_node,
            weight_type=_abi.SNN_W_BF16 if wl.weight_type == "bf16" else _abi.SNN_W_FP32,
            n_threads=n_threads, verbose=1 if verbose else 0, n_clusters=wl.n_clusters,
            p_in=wl.p_in)
        starts = synth.partition_starts(wl)
        fracs = synth.cross_fracs(wl)
        pm = None if part_map is None else np.ascontiguousarray(part_map, np.int32)
        h = _P()
        t0 = time.time()
        _abi.check(L.snn_setup_create(ctypes.byref(spec), None if starts is None else _ptr(starts),
                                      None if fracs is None else _ptr(fracs),
                                      None if pm is None else _ptr(pm), ctypes.byref(h)))
        try:
            sizes = [ctypes.c_uint64() for _ in range(4)]
            _abi.check(L.snn_setup_sizes(h, *[ctypes.byref(s) for s in sizes]))
            nnz = sizes[0].value
            N = wl.n_neurons
            if verbose:
                print(f"[setup] {wl.name}: counted {nnz:,} synapses in {time.time() - t0:.1f}s",
                      file=sys.stderr, flush=True)
            self.row_ptr = np.empty(N + 1, np.int64)
            self.n_local = np.empty(N, np.uint32)
            self.delay_off = np.empty(N * (wl.max_delay + 1), np.uint16)
            self.tgt_delay = np.empty(nnz, np.uint32)
            self.weight = np.empty(nnz, np.uint16 if wl.weight_type == "bf16" else np.float32)
            t1 = time.time()
            _abi.check(L.snn_setup_fill_rows(h, _ptr(self.row_ptr), _ptr(self.n_local),
                                             _ptr(self.delay_off), _ptr(self.tgt_delay),
                                             _ptr(self.weight)))
            _abi.check(L.snn_setup_sizes(h, *[ctypes.byref(s) for s in sizes]))
            pairs, self.bucket_total, self.recv_total = (s.value for s in sizes[1:])
            ib = ctypes.c_float()
            _abi.check(L.snn_setup_input_bound(h, ctypes.byref(ib)))
            self.input_bound = float(ib.value)
            if verbose:
                print(f"[setup] rows placed and sorted in {time.time() - t1:.1f}s; "
                      f"{pairs:,} destination pairs", file=sys.stderr, flush=True)
            n_nodes = wl.n_nodes
            self.vp_ptr = np.empty(N + 1, np.int64)
            self.vp_part = np.empty(max(pairs, 1), np.uint16)
            self.vp_rec = np.empty(2 * max(pairs, 1), np.uint64)
            self.part = np.empty(N, np.int32)
            self.bucket_off = np.empty(n_nodes + 1, np.uint64)
            self.recv_off = np.empty(wl.n_partitions + 1, np.uint64)
            _abi.check(L.snn_setup_fill_routes(h, _ptr(self.tgt_delay), _ptr(self.weight),
                                               _ptr(self.vp_ptr), _ptr(self.vp_part),
                                               _ptr(self.vp_rec), _ptr(self.part),
                                               _ptr(self.bucket_off), _ptr(self.recv_off)))
        finally:
            L.snn_setup_destroy(h)
        self.nnz, self.pairs = nnz, pairs
        self.setup_seconds = time.time() - t0

    def host_bytes(self) -> int:
        return sum(a.nbytes for a in (self.row_ptr, self.n_local, self.delay_off, self.tgt_delay,
                                      self.weight,
                                      self.vp_ptr, self.vp_part, self.vp_rec, self.part,
                                      self.bucket_off, self.recv_off))
