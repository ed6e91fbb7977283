"""MI355X-native per-GPU spiking-network step with two-level spike routing.

The hot path (neuron update + compaction, two-level / flat routing with mask
expansion, synaptic delivery) runs only in libsnn.so's HIP kernels for
gfx950, behind the C ABI of include/snn.h.  This package is the thin Python
binding over it: ``_abi`` mirrors the C declarations under the same names,
``network`` drives the host setup entry points, ``sim`` owns the device
tensors and the stream.  There is no CPU fallback: without libsnn.so (or
without a GPU) the calls raise.

``partition`` (Algorithm 1), ``grouping`` (Algorithm 2) and ``links``
(per-link traffic and bridge choice) are host-side setup and analysis in
numpy / scipy; they are imported on demand and run nothing on the GPU.
"""
from ._abi import (  # noqa: F401
    SNN_ROUTE_BOTH,
    SNN_ROUTE_FLAT,
    SNN_ROUTE_TWO_LEVEL,
    STAT_NAMES,
    SNNError,
    lib,
)
from .network import HostNetwork, derived_params  # noqa: F401


def Simulation(*args, **kwargs):
    from .sim import Simulation as _S
    return _S(*args, **kwargs)
