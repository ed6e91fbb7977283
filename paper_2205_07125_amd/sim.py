"""Device-side simulation handle: uploads a HostNetwork into torch tensors
(device memory owned by this object) and drives the C ABI on a torch stream.
Every step runs in libsnn's HIP kernels; this module only marshals."""
from __future__ import annotations

import ctypes

import numpy as np

from . import _abi
from .network import HostNetwork, default_caps, derived_params


def _dev(torch, a: np.ndarray, device):
    """Copy a host array to device memory, keeping its bit pattern (unsigned
    arrays travel as their signed twins)."""
    view = {np.uint32: np.int32, np.uint16: np.int16, np.uint64: np.int64}.get(a.dtype.type)
    if view is not None:
        a = a.view(view)
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


class Simulation:
    def __init__(self, wl, host: HostNetwork | None = None, device: str = "cuda",
                 log_steps: int | None = None, log_cap: int | None = None,
                 bucket_off=None, recv_off=None, bin_cap: int | None = None,
                 stage_cap: int | None = None, verbose: bool = False, static: bool = False,
                 tile_neurons: int = 0):
        """static: the handle comes from snn_create_static (workspace in the
        library's static device scratch, nothing allocated by the call; one such
        handle per device at a time, small networks only).  tile_neurons: neurons
        per tile (0: the library's default)."""
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the simulation runs only in libsnn's HIP kernels")
        _abi.lib()
        self.torch = torch
        self.wl = wl
        self.device = torch.device(device)
        host = host or HostNetwork(wl, verbose=verbose)
        self.host = host
        N = wl.n_neurons
        D = wl.max_delay + 1
        self.ring_stride = _abi.snn_ring_stride(N)
        if bucket_off is None:
            bucket_off = host.bucket_off
        if recv_off is None:
            recv_off = host.recv_off
        bucket_off = np.asarray(bucket_off, np.uint64)
        recv_off = np.asarray(recv_off, np.uint64)
        d = lambda a: _dev(torch, a, self.device)
        self.t_row_ptr = d(host.row_ptr)
        self.t_n_local = d(host.n_local)
        self.t_delay_off = d(host.delay_off)
        self.t_tgt_delay = d(host.tgt_delay)
        self.t_weight = d(host.weight)
        self.t_vp_ptr = d(host.vp_ptr)
        self.t_vp_part = d(host.vp_part)
        self.t_vp_rec = d(host.vp_rec)
        self.t_part = d(host.part)
        self.t_bucket_off = d(bucket_off)
        self.t_recv_off = d(recv_off)
        import synth
        self.u = d(synth.initial_u(wl))
        self.ref = torch.zeros(N, dtype=torch.uint8, device=self.device)
        self.ring = torch.zeros(D * self.ring_stride, dtype=torch.float32, device=self.device)

        dp = derived_params(wl)
        cb, cs = default_caps(wl, host, tile_neurons)
        self.tile_neurons = _abi.snn_bin_geometry(N, tile_neurons)[0]
        bin_cap = cb if bin_cap is None else bin_cap
        stage_cap = cs if stage_cap is None else stage_cap
        forced = bool(wl.forced)
        if log_steps is None:
            log_steps = max(wl.n_steps, 1)
        if log_cap is None:
            log_cap = min(N * 64, 1 << 26)
        self.params = _abi.snn_params(
            n_neurons=N, n_partitions=wl.n_partitions, gpus_per_node=wl.gpus_per_node,
            max_delay=wl.max_delay, alpha=dp["alpha"], theta=dp["theta"], u_reset=dp["u_reset"],
            w_ext=dp["w_ext"], n_ref=dp["n_ref"],
            poisson_thr=(ctypes.c_uint32 * 15)(*dp["poisson_thr"]), seed=wl.seed,
            weight_type=_abi.SNN_W_BF16 if wl.weight_type == "bf16" else _abi.SNN_W_FP32,
            flags=_abi.SNN_FORCED_RASTER if forced else 0,
            raster_thr_on=dp["raster_thr_on"], raster_thr_off=dp["raster_thr_off"],
            raster_period=max(wl.period_steps, 1), raster_on=wl.on_steps,
            bucket_total=int(bucket_off[-1]), recv_total=int(recv_off[-1]),
            log_steps=log_steps, input_bound=host.input_bound, log_cap=log_cap, bin_cap=bin_cap,
            stage_cap=stage_cap, tile_neurons=tile_neurons)
        self.ws_bytes = _abi.snn_workspace_size(self.params)
        self.static = static
        if not static:
            self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8,
                                         device=self.device)
            self.ws_ptr = (self.workspace.data_ptr() + 255) & ~255
        self.net = _abi.snn_network_dev(
            row_ptr=self.t_row_ptr.data_ptr(), n_local=self.t_n_local.data_ptr(),
            delay_off=self.t_delay_off.data_ptr(),
            tgt_delay=self.t_tgt_delay.data_ptr(), weight=self.t_weight.data_ptr(),
            vp_ptr=self.t_vp_ptr.data_ptr(), vp_part=self.t_vp_part.data_ptr(),
            vp_rec=self.t_vp_rec.data_ptr(), part_of_neuron=self.t_part.data_ptr(),
            bucket_off=self.t_bucket_off.data_ptr(), recv_off=self.t_recv_off.data_ptr(),
            u=self.u.data_ptr(), ref=self.ref.data_ptr(), ring=self.ring.data_ptr())
        # A stream of our own at default priority: graphs cannot be captured
        # on the legacy default stream.
        self.stream = torch.cuda.Stream(device=self.device)
        torch.cuda.synchronize(self.device)
        if static:
            self.h = _abi.snn_create_static(self.params, self.net, self.stream.cuda_stream)
        else:
            self.h = _abi.snn_create(self.params, self.net, self.ws_ptr, self.ws_bytes,
                                     self.stream.cuda_stream)

    # --- the C ABI, one call each -------------------------------------------------
    def step(self):
        _abi.snn_step(self.h)

    def route(self, mode=_abi.SNN_ROUTE_TWO_LEVEL):
        _abi.snn_route(self.h, mode)

    def step_route(self, mode=_abi.SNN_ROUTE_TWO_LEVEL):
        """snn_step_route: update and routing of one step in fewer launches."""
        _abi.snn_step_route(self.h, mode)

    def deliver(self):
        _abi.snn_deliver(self.h)

    def full_step(self, mode=_abi.SNN_ROUTE_TWO_LEVEL):
        self.step()
        self.route(mode)
        self.deliver()

    def run(self, n_steps: int, mode=_abi.SNN_ROUTE_TWO_LEVEL, use_graph=True):
        """use_graph: False eager, True 16-step graphs, 2 one graph of all n_steps."""
        _abi.snn_run(self.h, n_steps, mode, use_graph)

    def run_partitioned(self, n_steps: int, mode=_abi.SNN_ROUTE_TWO_LEVEL, use_graph=True):
        """snn_run_partitioned: the update launched once per partition (the
        workload's partitions must be contiguous ranges)."""
        import synth
        starts = synth.partition_starts(self.wl)
        if starts is None:     # loopback shapes: every neuron is in partition 0
            starts = np.full(self.wl.n_partitions + 1, self.wl.n_neurons, np.uint32)
            starts[0] = 0
        _abi.snn_run_partitioned(self.h, n_steps, mode, use_graph, starts)

    def set_tuning(self, update_blocks: int | None = None, recv_split: int | None = None,
                   recv_merged: int | None = None):
        """Sets the given launch shapes (snn_tuning); the others keep their values."""
        cur = self.tuning()
        new = {k: cur[k] if v is None else v for k, v in
               (("update_blocks", update_blocks), ("recv_split", recv_split),
                ("recv_merged", recv_merged))}
        _abi.snn_set_tuning(self.h, **new)

    def tuning(self) -> dict:
        return _abi.snn_get_tuning(self.h)

    def sync(self):
        _abi.snn_sync(self.h)

    def kernel_times(self, n_steps: int, mode=_abi.SNN_ROUTE_TWO_LEVEL) -> dict:
        """Runs n_steps steps with every kernel bracketed by HIP events on the
        simulation stream; -> {kernel name: average ms} (snn_kernel_times)."""
        ms = _abi.snn_kernel_times(self.h, n_steps, mode)
        return dict(zip(_abi.KERNEL_NAMES, ms))

    def flush(self):
        _abi.snn_flush(self.h)

    def ring_events(self) -> int:
        return _abi.snn_ring_events(self.h)

    @property
    def t(self) -> int:
        return _abi.snn_time(self.h)

    def read_spikes(self, first_step: int, n_steps: int):
        """-> (ids int32 concatenated, per-step counts uint32)."""
        L = _abi.lib()
        n = ctypes.c_uint64()
        counts = np.zeros(n_steps, np.uint32)
        _abi.check(L.snn_read_spikes(self.h, first_step, n_steps, None, 0,
                                     counts.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        ids = np.zeros(max(n.value, 1), np.int32)
        _abi.check(L.snn_read_spikes(self.h, first_step, n_steps,
                                     ids.ctypes.data_as(ctypes.c_void_p), ids.size,
                                     counts.ctypes.data_as(ctypes.c_void_p), ctypes.byref(n)))
        return ids[:n.value], counts

    def route_sizes(self, which: int) -> np.ndarray:
        """Entries per list (which 0 flat, 1 expanded, per partition) or
        messages per node bucket (which 2) of the last routed step, without
        copying the entries (snn_read_routes with entries = NULL)."""
        nl = self.wl.n_nodes if which == 2 else self.wl.n_partitions
        sizes = np.zeros(nl, np.uint64)
        n = ctypes.c_uint64()
        _abi.check(_abi.lib().snn_read_routes(self.h, which, sizes.ctypes.data_as(ctypes.c_void_p),
                                              None, 0, ctypes.byref(n)))
        return sizes

    def read_routes(self, which: int, sources_only: bool = False):
        """which 0 flat lists, 1 expanded lists (per partition): uint64 entries;
        2 node buckets (per node): (n, 2) uint64 messages (source | first pair
        index << 32, partition mask); see include/snn.h.  With sources_only,
        just the source ids."""
        L = _abi.lib()
        nl = self.wl.n_nodes if which == 2 else self.wl.n_partitions
        sizes = np.zeros(nl, np.uint64)
        n = ctypes.c_uint64()
        _abi.check(L.snn_read_routes(self.h, which, sizes.ctypes.data_as(ctypes.c_void_p), None, 0,
                                     ctypes.byref(n)))
        shape = (max(n.value, 1), 2) if which == 2 else (max(n.value, 1),)
        ent = np.zeros(shape, np.uint64)
        _abi.check(L.snn_read_routes(self.h, which, sizes.ctypes.data_as(ctypes.c_void_p),
                                     ent.ctypes.data_as(ctypes.c_void_p), shape[0], ctypes.byref(n)))
        if sources_only:
            if which == 2:
                ent = ent[:, 0]
            bits = _abi.ENTRY_SRC_BITS if which != 2 else 32
            ent = (ent & np.uint64((1 << bits) - 1)).astype(np.uint32)
        offs = np.concatenate([[0], np.cumsum(sizes.astype(np.int64))])
        return [ent[offs[i]:offs[i + 1]].copy() for i in range(nl)]

    def read_counters(self, first_step: int, n_steps: int) -> np.ndarray:
        out = np.zeros((n_steps, _abi.SNN_NSTAT), np.uint64)
        _abi.check(_abi.lib().snn_read_counters(self.h, first_step, n_steps,
                                                out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def membrane(self) -> np.ndarray:
        """u as a host array, after the stream's work; nothing else is read or
        moved, so the simulation continues exactly as it would have."""
        self.sync()
        return self.u.cpu().numpy()

    def state(self) -> dict:
        """u, ref and the ring (D x N) as host arrays: snn_flush writes the
        input scheduled for the coming steps into the ring first (reading
        only; later steps are unchanged)."""
        self.flush()
        self.sync()
        D, N = self.wl.max_delay + 1, self.wl.n_neurons
        ring = self.ring.view(D, self.ring_stride)[:, :N].cpu().numpy()
        return dict(u=self.u.cpu().numpy(), ref=self.ref.cpu().numpy(), ring=ring)

    def close(self):
        if getattr(self, "h", None):
            _abi.snn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
