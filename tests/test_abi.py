"""The C ABI library loads, exports every entry point the headers declare,
and rejects invalid arguments on the host (no kernel is launched)."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from paper_2205_07125_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in ("snn.h", "snn_setup.h"):
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"\b(snn_[a-z_0-9]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    lib = _abi.lib()
    declared = _declared()
    assert {"snn_create", "snn_step", "snn_route", "snn_deliver", "snn_read_spikes"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(_abi.EXPORTED)
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (snn_[a-z_0-9]+)", out))
    assert declared <= exported


def test_library_has_gfx950_code():
    blob = open(_abi.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def _params(**kw):
    p = _abi.snn_params(n_neurons=1000, n_partitions=8, gpus_per_node=4, max_delay=10,
                        alpha=0.995, theta=15.0, u_reset=0.0, w_ext=0.1, n_ref=20, seed=1,
                        raster_period=1, bucket_total=100, recv_total=100, log_steps=10,
                        input_bound=100.0, log_cap=1000)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_workspace_size_and_ring_stride():
    assert _abi.snn_ring_stride(1) == 256 and _abi.snn_ring_stride(256) == 256
    assert _abi.snn_ring_stride(5_000_000) % 256 == 0
    a = _abi.snn_workspace_size(_params())
    b = _abi.snn_workspace_size(_params(recv_total=10_000))
    assert b - a >= 2 * 4 * 9_900   # flat and expanded lists
    assert a % 256 == 0


@pytest.mark.parametrize("field,value", [
    ("n_neurons", 0), ("n_neurons", (1 << 27) + 1), ("n_partitions", 0),
    ("n_partitions", 65536), ("gpus_per_node", 0), ("gpus_per_node", 65), ("max_delay", 0),
    ("max_delay", 16), ("n_ref", 256), ("weight_type", 2), ("flags", 2), ("log_steps", 0),
    ("input_bound", 0.0), ("input_bound", -1.0), ("input_bound", float("nan")),
    ("input_bound", float("inf")),
])
def test_invalid_params_rejected(field, value):
    with pytest.raises(_abi.SNNError) as ei:
        _abi.snn_workspace_size(_params(**{field: value}))
    assert ei.value.status == _abi.SNN_ERR_INVALID_ARG
    assert _abi.snn_last_error()


def test_input_bound_too_large_unsupported():
    # more than 2^22 mV per step would leave fewer than 8 fractional bits
    with pytest.raises(_abi.SNNError) as ei:
        _abi.snn_workspace_size(_params(input_bound=float(1 << 23)))
    assert ei.value.status == _abi.SNN_ERR_UNSUPPORTED
    assert _abi.snn_workspace_size(_params(input_bound=float(1 << 21))) > 0


def test_bin_geometry():
    tile, deliver_blocks, stage_blocks = _abi.snn_bin_geometry(5_000_000)
    assert deliver_blocks > 0 and stage_blocks % deliver_blocks == 0
    # default: 8192, or the neurons spread over 512 tiles (rounded up to 64, at least 2048)
    assert tile == 8192
    assert _abi.snn_bin_geometry(5_800_000)[0] == 8192
    assert _abi.snn_bin_geometry(1_000_000)[0] == 2048
    assert _abi.snn_bin_geometry(3_000_000)[0] == 5888 and -(-3_000_000 // 5888) <= 512
    assert _abi.snn_bin_geometry(1_000)[0] == 2048
    assert _abi.snn_bin_geometry(1_000, 64)[0] == 64
    assert _abi.snn_bin_geometry(100_000_000)[0] == 8192
    assert _abi.snn_bin_geometry(5_000_000, 8192)[0] == 8192
    for bad in (100, 8256, 16384):
        with pytest.raises(_abi.SNNError):
            _abi.snn_bin_geometry(5_000_000, bad)


def test_tile_divider_formula():
    """floor(x / T) as umulhi(x, M) >> (c - 1), M = ceil(2^(31+c) / T), c =
    ceil(log2 T): exact for every neuron id below 2^27 (checked at the
    multiples of T and their neighbours, where an error would show first, and
    at random ids)."""
    rng = np.random.default_rng(3)
    for t in list(range(64, 8193, 64)):
        c = (t - 1).bit_length()
        m = -(-(1 << (31 + c)) // t)
        assert m < 1 << 32
        q = np.arange(0, (1 << 27) // t + 2, dtype=np.uint64)
        x = np.concatenate([q * t, q * t + t - 1, q * t - 1, rng.integers(0, 1 << 27, 4096,
                                                                        dtype=np.uint64)])
        x = x[(x < (1 << 27))]
        got = ((x * np.uint64(m)) >> np.uint64(32)) >> np.uint64(c - 1)
        assert np.array_equal(got, x // np.uint64(t)), t


def test_nonmonotone_poisson_table_rejected():
    p = _params()
    p.poisson_thr[3] = 10
    p.poisson_thr[4] = 5
    with pytest.raises(_abi.SNNError):
        _abi.snn_workspace_size(p)


def test_create_rejects_null_arrays_and_bad_workspace():
    p = _params()
    net = _abi.snn_network_dev()
    with pytest.raises(_abi.SNNError) as ei:
        _abi.snn_create(p, net, 0, 0, 0)
    assert ei.value.status == _abi.SNN_ERR_INVALID_ARG
    assert "row_ptr" in _abi.snn_last_error()
    # every array present (fake, never dereferenced), workspace misaligned
    fake = {n: 4096 * (i + 1) for i, (n, _) in enumerate(_abi.snn_network_dev._fields_)}
    net = _abi.snn_network_dev(**fake)
    with pytest.raises(_abi.SNNError) as ei:
        _abi.snn_create(p, net, 4096 + 8, 1 << 30, 0)
    assert "aligned" in _abi.snn_last_error()
    with pytest.raises(_abi.SNNError):
        _abi.snn_create(p, net, 4096, 16, 0)   # too small


def test_create_static_rejects_before_touching_the_device():
    """Argument errors and a workspace larger than the static scratch are
    reported on the host, before any HIP call."""
    p = _params()
    with pytest.raises(_abi.SNNError) as ei:
        _abi.snn_create_static(p, _abi.snn_network_dev(), 0)
    assert ei.value.status == _abi.SNN_ERR_INVALID_ARG
    fake = {n: 4096 * (i + 1) for i, (n, _) in enumerate(_abi.snn_network_dev._fields_)}
    net = _abi.snn_network_dev(**fake)
    big = _params()
    big.recv_total = _abi.SNN_STATIC_SCRATCH_BYTES // 8     # the lists alone fill the scratch
    assert _abi.snn_workspace_size(big) > _abi.SNN_STATIC_SCRATCH_BYTES
    with pytest.raises(_abi.SNNError) as ei:
        _abi.snn_create_static(big, net, 0)
    assert ei.value.status == _abi.SNN_ERR_UNSUPPORTED
    assert "static scratch" in _abi.snn_last_error()


def test_null_handle_calls():
    L = _abi.lib()
    assert L.snn_step(None) == _abi.SNN_ERR_INVALID_ARG
    assert L.snn_route(None, 0) == _abi.SNN_ERR_INVALID_ARG
    assert L.snn_deliver(None) == _abi.SNN_ERR_INVALID_ARG
    assert L.snn_destroy(None) == _abi.SNN_OK
    n = ctypes.c_uint64()
    assert L.snn_read_spikes(None, 0, 1, None, 0, None, ctypes.byref(n)) == _abi.SNN_ERR_INVALID_ARG
    out = (ctypes.c_float * _abi.SNN_NKERNEL)()
    assert L.snn_kernel_times(None, 1, 0, out) == _abi.SNN_ERR_INVALID_ARG


def test_counter_and_kernel_enums_match_binding():
    """The binding's counter and kernel-kind names follow the header's enum order."""
    src = open(os.path.join(ROOT, "include", "snn.h")).read()
    stats = dict((m[0], int(m[1])) for m in re.findall(r"SNN_STAT_([A-Z0-9_]+) = (\d+)", src))
    assert [k.lower() for k, _ in sorted(stats.items(), key=lambda kv: kv[1])] == _abi.STAT_NAMES
    kinds = dict((m[0], int(m[1])) for m in re.findall(r"SNN_KERNEL_([A-Z0-9_]+) = (\d+)", src))
    assert [k.lower() for k, _ in sorted(kinds.items(), key=lambda kv: kv[1])] == _abi.KERNEL_NAMES
    assert int(re.search(r"SNN_NKERNEL = (\d+)", src).group(1)) == _abi.SNN_NKERNEL
    assert int(re.search(r"SNN_NSTAT = (\d+)", src).group(1)) == _abi.SNN_NSTAT


def test_static_scratch_size_matches_header():
    src = open(os.path.join(ROOT, "include", "snn.h")).read()
    m = re.search(r"#define SNN_STATIC_SCRATCH_BYTES \((\d+)u << (\d+)\)", src)
    assert m and int(m.group(1)) << int(m.group(2)) == _abi.SNN_STATIC_SCRATCH_BYTES


def test_one_hip_runtime_in_process():
    """Loading the library leaves exactly one libamdhip64 mapped (torch's):
    two runtimes in one process find no device."""
    code = ("from paper_2205_07125_amd import _abi; _abi.lib(); "
            "m = open('/proc/self/maps').read(); "
            "print(len({l.split()[-1] for l in m.splitlines() if 'libamdhip64' in l}))")
    out = subprocess.run([os.sys.executable, "-c", code], cwd=ROOT, capture_output=True,
                         text=True, check=True).stdout
    assert out.strip() == "1"
