// snn_internal.h — device-side state and kernel parameter block shared by the
// kernels and the host runtime of libsnn.  Not part of the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "snn.h"

namespace snn {

// Sticky device error bits (DevState::error).
enum : uint32_t {
  ERR_BUCKET = 1u,   // a node's send bucket overflowed
  ERR_RECV = 2u,     // an expanded receive list overflowed
  ERR_FLAT = 4u,     // a flat receive list overflowed
  ERR_LOG = 8u,      // a step had more spikes than the spike log holds
  ERR_ROUTE = 16u    // a receive entry names a source without that partition
};

// Device-resident step state.  Every step-dependent value lives here so that
// a captured step replays unchanged.
struct DevState {
  uint64_t t;          // step the next update kernel runs
  uint64_t log_total;  // ids appended to the spike log so far
  uint32_t n_fired;    // spikes of the step in flight (t - 1 after the update)
  uint32_t error;      // sticky ERR_* bits
  uint32_t pad[10];
};

// Stream ids of the counter-based generator.
enum : uint32_t { STREAM_POISSON = 1u, STREAM_RASTER = 2u };

// Kernel launch geometry.
constexpr int UPDATE_THREADS = 256;
constexpr int UPDATE_NPT_MIN = 4;   // neurons per thread: 4, 8 or 16 (tuning knob)
constexpr int ROUTE_THREADS = 256;
constexpr int DELIVER_THREADS = 256;

// Everything a kernel needs, passed by value.
struct KParams {
  // model
  uint32_t N, P, G, D, n_nodes;
  uint32_t n_ref;
  uint64_t ring_stride;
  float alpha, theta, u_reset, w_ext;
  uint32_t thr[15];
  uint32_t seed_lo, seed_hi;
  uint32_t forced, raster_on_thr, raster_off_thr, raster_period, raster_on;
  uint32_t bf16;
  uint32_t log_steps;
  uint64_t log_cap;
  // network (caller-owned device memory)
  const int64_t* row_ptr;
  const uint32_t* n_local;
  const uint32_t* tgt_delay;
  const void* weight;
  const int64_t* vp_ptr;
  const uint16_t* vp_part;
  const uint32_t* vp_seg;
  const int32_t* part;
  const uint64_t* bucket_off;
  const uint64_t* recv_off;
  float* u;
  uint8_t* ref;
  float* ring;
  // workspace
  DevState* st;
  uint64_t* lookback;   // [update blocks] decoupled look-back words
  uint32_t* fired;      // [N] ascending fired ids of the step in flight
  uint32_t* bucket_cnt; // [n_nodes]
  uint64_t* bucket;     // [bucket_total]
  uint32_t* recv_cnt;   // [P] expanded lists
  uint32_t* recv;       // [recv_total]
  uint32_t* flat_cnt;   // [P]
  uint32_t* flat;       // [recv_total]
  uint64_t* stats;      // [log_steps][SNN_NSTAT]
  uint64_t* log_off;    // [log_steps] first log position of each step
  uint32_t* log;        // [log_cap] spike-log ring
};

// Launchers (snn_kernels.hip); all enqueue on `s` and return the launch error.
uint32_t update_blocks(uint32_t n, int npt);
hipError_t launch_update(const KParams& p, int npt, hipStream_t s);
hipError_t launch_route(const KParams& p, int mode, hipStream_t s);
hipError_t launch_deliver(const KParams& p, int mode, hipStream_t s);

}  // namespace snn
