// snn_runtime.hip — host side of the C ABI declared in include/snn.h:
// parameter validation, workspace carve-up, the step -> route -> deliver
// state machine, HIP-graph replay of whole steps, and read-back.
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "snn_internal.h"

using namespace snn;


namespace {
thread_local char g_err[512] = "";
}

// Records the message returned by snn_last_error; shared with the host
// setup code of the same library (not exported).
extern "C" __attribute__((visibility("hidden"))) snn_status snn_fail_v(snn_status s,
                                                                       const char* fmt,
                                                                       va_list ap) {
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  return s;
}

namespace {

snn_status fail(snn_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  snn_fail_v(s, fmt, ap);
  va_end(ap);
  return s;
}

#define HIP_TRY(call)                                                                    \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return fail(SNN_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

uint32_t n_nodes_of(const snn_params* p) {
  return (p->n_partitions + p->gpus_per_node - 1) / p->gpus_per_node;
}

// Byte offsets of the workspace regions.
struct Layout {
  uint64_t st, tickets, sync, ovf, lookback, fired, bucket_cnt, bucket, recv_cnt, recv, flat_cnt, flat,
      stage_cnt, stage, bin_cnt, dirty, bins, stats, pois_lut, log_off, log, total;
};

Layout layout(const snn_params* p) {
  Layout L{};
  uint64_t o = 0;
  auto take = [&](uint64_t bytes) {
    uint64_t at = o;
    o = align256(o + bytes);
    return at;
  };
  const uint32_t T = tile_size(p->n_neurons, p->tile_neurons);
  const uint64_t D = p->max_delay + 1, md = p->max_delay, tiles = (p->n_neurons + T - 1) / T;
  L.st = take(sizeof(DevState));
  L.tickets = take(sizeof(uint32_t) * 2);
  L.sync = take(sizeof(uint32_t) * SYNC_WORDS);
  L.ovf = take(sizeof(int32_t) * D * snn_ring_stride(p->n_neurons));
  L.lookback = take(sizeof(uint64_t) * tiles);
  L.fired = take(sizeof(uint32_t) * uint64_t(p->n_neurons));
  L.bucket_cnt = take(2 * sizeof(uint32_t) * CNT_STRIDE * n_nodes_of(p));
  L.recv_cnt = take(sizeof(uint32_t) * CNT_STRIDE * p->n_partitions);
  L.flat_cnt = take(sizeof(uint32_t) * CNT_STRIDE * p->n_partitions);
  L.stage_cnt = take(sizeof(uint32_t) * md * STAGE_BLOCKS);
  L.bin_cnt = take(sizeof(uint32_t) * D * tiles * md * DELIVER_BLOCKS);
  L.dirty = take(sizeof(uint32_t) * D * tiles);
  L.stats = take(sizeof(uint64_t) * STAT_ROW_WORDS * (uint64_t(p->log_steps) + 1));
  L.pois_lut = take(POIS_LUT_SIZE);
  L.log_off = take(sizeof(uint64_t) * uint64_t(p->log_steps));
  // large buffers last: the region before them is zeroed at create
  L.bucket = take(2 * sizeof(uint64_t) * p->bucket_total);
  L.recv = take(sizeof(uint64_t) * p->recv_total);
  L.flat = take(sizeof(uint64_t) * p->recv_total);
  L.stage = take(sizeof(Event) * md * STAGE_BLOCKS * p->stage_cap);
  L.bins = take(sizeof(Event) * D * tiles * md * DELIVER_BLOCKS * p->bin_cap);
  L.log = take(sizeof(uint32_t) * p->log_cap);
  L.total = o;
  return L;
}

// Poisson inversion lookup (layout in snn_internal.h): for the draws of entry
// b, [lo, hi], k = #{j : thr[j] <= r} is fixed when no threshold lies in
// (lo, hi]; one threshold there is resolved by one comparison in the kernel.
void build_pois_lut(const uint32_t* thr, uint8_t* lut) {
  for (uint32_t b = 0; b < POIS_LUT_SIZE; ++b) {
    const uint64_t lo = uint64_t(b) << POIS_LUT_SHIFT;
    const uint64_t hi = lo + (uint64_t(1) << POIS_LUT_SHIFT) - 1;
    uint32_t k_lo = 0, k_hi = 0;
    for (int j = 0; j < 15; ++j) {
      k_lo += thr[j] <= lo ? 1u : 0u;
      k_hi += thr[j] <= hi ? 1u : 0u;
    }
    lut[b] = k_hi == k_lo ? uint8_t(k_lo) : k_hi == k_lo + 1 ? uint8_t(16 + k_lo) : POIS_LUT_SLOW;
  }
}

// Fractional bits of the fixed-point input sums: the largest F <= 30 with
// input_bound * 2^F <= 2^30, which leaves 2^30 of headroom in int32 for the
// rounding of each weight to a multiple of 2^-F.
int input_shift(float bound) {
  int f = 30;
  while (f > 0 && std::ldexp(double(bound), f) > std::ldexp(1.0, 30)) --f;
  return f;
}

snn_status check_tile(const snn_params* p) {
  if (p->n_neurons == 0 || p->n_neurons > SNN_MAX_NEURONS)
    return fail(SNN_ERR_INVALID_ARG, "n_neurons=%u outside [1, 2^27]", p->n_neurons);
  const uint32_t t = p->tile_neurons;
  if (t && (t % TILE_ALIGN || t > TILE_MAX))
    return fail(SNN_ERR_INVALID_ARG, "tile_neurons=%u is not a multiple of %u in [%u, %u]", t,
                TILE_ALIGN, TILE_ALIGN, TILE_MAX);
  return SNN_OK;
}

snn_status check_params(const snn_params* p) {
  if (!p) return fail(SNN_ERR_INVALID_ARG, "params is NULL");
  snn_status st = check_tile(p);
  if (st != SNN_OK) return st;
  if (p->n_partitions == 0 || p->n_partitions > SNN_MAX_PARTITIONS)
    return fail(SNN_ERR_INVALID_ARG, "n_partitions=%u outside [1, 65535]", p->n_partitions);
  if (p->gpus_per_node == 0 || p->gpus_per_node > SNN_MAX_GPUS_PER_NODE)
    return fail(SNN_ERR_INVALID_ARG, "gpus_per_node=%u outside [1, %u]", p->gpus_per_node,
                SNN_MAX_GPUS_PER_NODE);
  if (p->max_delay == 0 || p->max_delay > SNN_MAX_DELAY)
    return fail(SNN_ERR_INVALID_ARG, "max_delay=%u outside [1, 15]", p->max_delay);
  if (p->n_ref > 255) return fail(SNN_ERR_INVALID_ARG, "n_ref=%u > 255", p->n_ref);
  for (int j = 1; j < 15; ++j)
    if (p->poisson_thr[j] < p->poisson_thr[j - 1])
      return fail(SNN_ERR_INVALID_ARG, "poisson_thr is not nondecreasing at %d", j);
  if (p->weight_type != SNN_W_FP32 && p->weight_type != SNN_W_BF16)
    return fail(SNN_ERR_INVALID_ARG, "weight_type=%u", p->weight_type);
  if (p->flags & ~uint32_t(SNN_FORCED_RASTER))
    return fail(SNN_ERR_INVALID_ARG, "unknown flags 0x%x", p->flags);
  if ((p->flags & SNN_FORCED_RASTER) && p->raster_period == 0)
    return fail(SNN_ERR_INVALID_ARG, "raster_period must be >= 1");
  if (p->log_steps == 0) return fail(SNN_ERR_INVALID_ARG, "log_steps must be >= 1");
  if (p->bin_cap > 0xFFFFFFFFull || p->stage_cap > 0xFFFFFFFFull)
    return fail(SNN_ERR_INVALID_ARG, "bin_cap and stage_cap must fit 32 bits");
  if (!(p->input_bound > 0.f) || !std::isfinite(p->input_bound))
    return fail(SNN_ERR_INVALID_ARG, "input_bound must be a positive finite number");
  const int f = input_shift(p->input_bound);
  if (f < 8)
    return fail(SNN_ERR_UNSUPPORTED, "input_bound %g mV leaves fewer than 8 fractional bits",
                double(p->input_bound));
  return SNN_OK;
}

}  // namespace

struct snn_ctx {
  snn_params prm;
  snn_network_dev net;
  hipStream_t stream;
  KParams kp;
  int phase;          // 0: expects step, 1: route, 2: deliver
  int route_mode;     // mode of the step in flight
  bool expand_deferred;  // snn_step_route left the mask expansion to snn_deliver
  uint64_t t_host;    // steps enqueued
  uint64_t handoff_t;  // step counter read by the last one-launch receive side (0: none)
  uint64_t routed_t;  // step whose routes are in the buffers (+1), 0 = none
  // captured steps, per layout (0: one update launch per step, 1: one per
  // partition) and route mode: one step, GRAPH_STEPS steps
  hipGraphExec_t graph[2][3][2];
  hipGraphExec_t whole;         // all steps of one snn_run call (use_graph = 2)
  uint32_t whole_key[3];        // its steps, mode, layout
  std::vector<uint32_t> part_start;   // partition starts of the per-partition layout
  uint8_t pois_lut[POIS_LUT_SIZE];  // host copy of the lookup uploaded at create
  bool is_static;     // from snn_create_static: lives in static storage, never freed
};

// Steps captured in the long graph: replaying several steps per launch spreads
// the graph launch cost (several microseconds) over them.
constexpr uint32_t GRAPH_STEPS = 16;

// The one-launch receive side tags its hand-off flags with the low 28 bits of
// the step counter it reads, which is t_host + 1 during step t_host.  The
// flags keep the tag of the last such launch (0 in a new workspace), so a
// launch a nonzero multiple of 2^28 steps later, with none in between, would
// take them as current.  The runtime gives that one step the three-launch
// receive side (same results, flags left alone); the steps after it differ
// from the stored tag again.
constexpr uint64_t HANDOFF_TAG_MASK = (uint64_t(1) << 28) - 1;

static bool handoff_tag_repeats(const snn_ctx* h) {
  const uint64_t t = h->t_host + 1;
  return t != h->handoff_t && ((t - h->handoff_t) & HANDOFF_TAG_MASK) == 0;
}

// The receive side of a whole step in `mode` runs as one launch.
static bool handoff_used(const snn_ctx* h, int mode) {
  return mode != SNN_ROUTE_FLAT && h->kp.recv_merged;
}

// Scratch of the allocation-free entry point (snn_create_static): the whole
// workspace of one handle, at most SNN_STATIC_SCRATCH_BYTES.  Each device that
// runs the library holds its own copy until the process ends.  Host code
// never passes the array's name as an address: each device's copy is found
// with hipGetSymbolAddress, that device current, and kept in g_scratch.
__device__ __align__(256) uint8_t scratch[SNN_STATIC_SCRATCH_BYTES];

namespace {
constexpr int STATIC_DEVICES = 64;
void* g_scratch[STATIC_DEVICES];        // device address of each device's copy of scratch
snn_ctx g_static_ctx[STATIC_DEVICES];   // the handle that uses it
}  // namespace

extern "C" {

uint64_t snn_ring_stride(uint32_t n_neurons) { return (uint64_t(n_neurons) + 255) & ~uint64_t(255); }

const char* snn_last_error(void) { return g_err; }

snn_status snn_workspace_size(const snn_params* params, size_t* bytes) {
  snn_status s = check_params(params);
  if (s != SNN_OK) return s;
  if (!bytes) return fail(SNN_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = layout(params).total;
  return SNN_OK;
}

namespace {

snn_status check_net(const snn_network_dev* net) {
  if (!net) return fail(SNN_ERR_INVALID_ARG, "net is NULL");
  const void* req[] = {net->row_ptr, net->n_local, net->delay_off, net->tgt_delay, net->weight,
                       net->vp_ptr, net->vp_part, net->vp_rec, net->part_of_neuron,
                       net->bucket_off, net->recv_off, net->u, net->ref, net->ring};
  const char* names[] = {"row_ptr", "n_local", "delay_off", "tgt_delay", "weight", "vp_ptr",
                         "vp_part", "vp_rec", "part_of_neuron", "bucket_off", "recv_off", "u",
                         "ref", "ring"};
  for (int i = 0; i < 14; ++i)
    if (!req[i]) return fail(SNN_ERR_INVALID_ARG, "net->%s is NULL", names[i]);
  if ((reinterpret_cast<uintptr_t>(net->u) & 15) || (reinterpret_cast<uintptr_t>(net->ring) & 15) ||
      (reinterpret_cast<uintptr_t>(net->ref) & 3))
    return fail(SNN_ERR_INVALID_ARG, "u and ring must be 16-byte aligned, ref 4-byte aligned");
  return SNN_OK;
}

// Fills c for params / net with its workspace at ws (layout L) and clears
// the workspace's counters on the stream.  device_setup: the clearing and the
// Poisson lookup are kernels, so the stream gets no memset node and no copy
// from host memory.
snn_status init_ctx(snn_ctx* c, const snn_params* params, const snn_network_dev* net, char* ws,
                    const Layout& L, void* stream, bool device_setup) {
  c->prm = *params;
  c->net = *net;
  c->stream = static_cast<hipStream_t>(stream);
  KParams& k = c->kp;
  k.N = params->n_neurons;
  k.P = params->n_partitions;
  k.G = params->gpus_per_node;
  // node of partition v: v * ceil(2^32 / G) >> 32 for G >= 2 (exact for v < 2^16)
  k.g_magic = k.G >= 2 ? static_cast<uint32_t>(((uint64_t(1) << 32) + k.G - 1) / k.G) : 0u;
  k.D = params->max_delay + 1;
  k.n_nodes = n_nodes_of(params);
  k.tile = tile_size(params->n_neurons, params->tile_neurons);
  tile_divider(k.tile, &k.tile_magic, &k.tile_shift);
  k.n_tiles = (params->n_neurons + k.tile - 1) / k.tile;
  k.tile0 = 0;
  k.tile_end = k.n_tiles;
  k.lo = 0;
  k.hi = k.N;
  k.step_ends = 1;
  k.recv_merged = 1;   // the receive side as one launch (snn_tuning)
  k.n_ref = params->n_ref;
  k.ring_stride = snn_ring_stride(params->n_neurons);
  k.alpha = params->alpha;
  k.theta = params->theta;
  k.u_reset = params->u_reset;
  k.w_ext = params->w_ext;
  std::memcpy(k.thr, params->poisson_thr, sizeof(k.thr));
  k.seed_lo = uint32_t(params->seed);
  k.seed_hi = uint32_t(params->seed >> 32);
  k.forced = (params->flags & SNN_FORCED_RASTER) ? 1u : 0u;
  k.raster_on_thr = params->raster_thr_on;
  k.raster_off_thr = params->raster_thr_off;
  k.raster_period = params->raster_period ? params->raster_period : 1u;
  k.raster_on = params->raster_on;
  k.bf16 = params->weight_type == SNN_W_BF16 ? 1u : 0u;
  k.log_steps = params->log_steps;
  k.log_cap = params->log_cap;
  k.bin_cap = params->bin_cap;
  const int wq_shift = input_shift(params->input_bound);
  k.wq_scale = std::ldexp(1.0f, wq_shift);
  k.wq_inv = std::ldexp(1.0, -wq_shift);
  k.stage_cap = params->stage_cap;
  k.row_ptr = net->row_ptr;
  k.n_local = net->n_local;
  k.delay_off = net->delay_off;
  k.tgt_delay = net->tgt_delay;
  k.weight = net->weight;
  k.vp_ptr = net->vp_ptr;
  k.vp_part = net->vp_part;
  k.vp_rec = net->vp_rec;
  k.part = net->part_of_neuron;
  k.bucket_off = net->bucket_off;
  k.recv_off = net->recv_off;
  k.u = net->u;
  k.ref = net->ref;
  k.ring = net->ring;
  k.st = reinterpret_cast<DevState*>(ws + L.st);
  k.lookback = reinterpret_cast<uint64_t*>(ws + L.lookback);
  k.tickets = reinterpret_cast<uint32_t*>(ws + L.tickets);
  k.sync = reinterpret_cast<uint32_t*>(ws + L.sync);
  k.ovf = reinterpret_cast<int32_t*>(ws + L.ovf);
  k.fired = reinterpret_cast<uint32_t*>(ws + L.fired);
  k.bucket_cnt = reinterpret_cast<uint32_t*>(ws + L.bucket_cnt);
  k.bucket = reinterpret_cast<uint64_t*>(ws + L.bucket);
  k.recv_cnt = reinterpret_cast<uint32_t*>(ws + L.recv_cnt);
  k.recv = reinterpret_cast<uint64_t*>(ws + L.recv);
  k.flat_cnt = reinterpret_cast<uint32_t*>(ws + L.flat_cnt);
  k.flat = reinterpret_cast<uint64_t*>(ws + L.flat);
  k.stage_cnt = reinterpret_cast<uint32_t*>(ws + L.stage_cnt);
  k.stage = reinterpret_cast<Event*>(ws + L.stage);
  k.bin_cnt = reinterpret_cast<uint32_t*>(ws + L.bin_cnt);
  k.dirty = reinterpret_cast<uint32_t*>(ws + L.dirty);
  k.bins = reinterpret_cast<Event*>(ws + L.bins);
  k.stats = reinterpret_cast<uint64_t*>(ws + L.stats);
  k.pois_lut = reinterpret_cast<const uint8_t*>(ws + L.pois_lut);
  k.log_off = reinterpret_cast<uint64_t*>(ws + L.log_off);
  k.log = reinterpret_cast<uint32_t*>(ws + L.log);
  // Everything before the large buffers starts at zero: state, look-back
  // words, counters (bin counts are read before their first write).
  // totals of the network arrays, for the kernels' bounds checks
  int64_t tot[2] = {0, 0};
  hipError_t e = hipMemcpy(&tot[0], net->vp_ptr + params->n_neurons, 8, hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(&tot[1], net->row_ptr + params->n_neurons, 8, hipMemcpyDeviceToHost);
  if (e != hipSuccess)
    return fail(SNN_ERR_HIP, "create: reading vp_ptr[N], row_ptr[N]: %s", hipGetErrorString(e));
  if (tot[0] < 0 || tot[1] < 0 || tot[1] >= (int64_t(1) << 40) || tot[0] >= (int64_t(1) << 32))
    return fail(SNN_ERR_INVALID_ARG,
                "vp_ptr[N] = %lld (< 2^32 required: messages carry 32-bit pair indices) or "
                "row_ptr[N] = %lld (< 2^40) out of range",
                (long long)tot[0], (long long)tot[1]);
  k.n_pairs = uint64_t(tot[0]);
  k.nnz = uint64_t(tot[1]);
  if (device_setup) {
    e = launch_zero(ws, L.bucket, c->stream);
    if (e == hipSuccess)
      e = launch_pois_lut(k, reinterpret_cast<uint8_t*>(ws + L.pois_lut), c->stream);
  } else {
    e = hipMemsetAsync(ws, 0, L.bucket, c->stream);
    build_pois_lut(params->poisson_thr, c->pois_lut);
    if (e == hipSuccess)
      e = hipMemcpyAsync(ws + L.pois_lut, c->pois_lut, POIS_LUT_SIZE, hipMemcpyHostToDevice,
                         c->stream);
  }
  if (e == hipSuccess) {
    e = prepare_kernels(k);
    if (e == hipErrorInvalidConfiguration)
      return fail(SNN_ERR_UNSUPPORTED,
                  "create: %u tiles of neurons leave no deliver window in the device's LDS "
                  "(about 8e7 neurons at most)", k.n_tiles);
  }
  if (e != hipSuccess) return fail(SNN_ERR_HIP, "create: %s", hipGetErrorString(e));
  return SNN_OK;
}

}  // namespace

snn_status snn_create(const snn_params* params, const snn_network_dev* net, void* workspace,
                      size_t workspace_bytes, void* stream, snn_handle* out) {
  if (!out) return fail(SNN_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  snn_status s = check_params(params);
  if (s != SNN_OK) return s;
  s = check_net(net);
  if (s != SNN_OK) return s;
  const Layout L = layout(params);
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) & 255))
    return fail(SNN_ERR_INVALID_ARG, "workspace must be non-NULL and 256-byte aligned");
  if (workspace_bytes < L.total)
    return fail(SNN_ERR_INVALID_ARG, "workspace has %zu bytes, needs %llu", workspace_bytes,
                (unsigned long long)L.total);
  snn_ctx* c = new snn_ctx();
  s = init_ctx(c, params, net, static_cast<char*>(workspace), L, stream, false);
  if (s != SNN_OK) {
    delete c;
    return s;
  }
  *out = c;
  return SNN_OK;
}

snn_status snn_create_static(const snn_params* params, const snn_network_dev* net, void* stream,
                             snn_handle* out) {
  if (!out) return fail(SNN_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  snn_status s = check_params(params);
  if (s != SNN_OK) return s;
  s = check_net(net);
  if (s != SNN_OK) return s;
  const Layout L = layout(params);
  if (L.total > SNN_STATIC_SCRATCH_BYTES)
    return fail(SNN_ERR_UNSUPPORTED,
                "snn_create_static: the network needs %llu bytes of workspace, more than the "
                "%u bytes of the static scratch; use snn_create with a workspace",
                (unsigned long long)L.total, SNN_STATIC_SCRATCH_BYTES);
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= STATIC_DEVICES)
    return fail(SNN_ERR_UNSUPPORTED, "snn_create_static: device %d (at most %d devices)", dev,
                STATIC_DEVICES);
  if (!g_scratch[dev]) {
    // once per device, with that device current: the address of its copy
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(SNN_ERR_HIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch[dev] = ptr;
  }
  snn_ctx* c = &g_static_ctx[dev];
  *c = snn_ctx{};
  c->is_static = true;
  s = init_ctx(c, params, net, static_cast<char*>(g_scratch[dev]), L, stream, true);
  if (s != SNN_OK) {
    *c = snn_ctx{};
    return s;
  }
  *out = c;
  return SNN_OK;
}

snn_status snn_step(snn_handle h) {
  if (!h) return fail(SNN_ERR_INVALID_ARG, "handle is NULL");
  if (h->phase != 0) return fail(SNN_ERR_BAD_STATE, "snn_step called before snn_deliver");
  HIP_TRY(launch_update(h->kp, h->stream));
  h->phase = 1;
  return SNN_OK;
}

snn_status snn_route(snn_handle h, int mode) {
  if (!h) return fail(SNN_ERR_INVALID_ARG, "handle is NULL");
  if (mode < SNN_ROUTE_TWO_LEVEL || mode > SNN_ROUTE_BOTH)
    return fail(SNN_ERR_INVALID_ARG, "route mode %d", mode);
  if (h->phase != 1) return fail(SNN_ERR_BAD_STATE, "snn_route must follow snn_step");
  HIP_TRY(launch_route(h->kp, mode, h->stream));
  h->route_mode = mode;
  h->phase = 2;
  h->routed_t = h->t_host + 1;
  return SNN_OK;
}

snn_status snn_step_route(snn_handle h, int mode) {
  if (!h) return fail(SNN_ERR_INVALID_ARG, "handle is NULL");
  if (mode < SNN_ROUTE_TWO_LEVEL || mode > SNN_ROUTE_BOTH)
    return fail(SNN_ERR_INVALID_ARG, "route mode %d", mode);
  if (h->phase != 0) return fail(SNN_ERR_BAD_STATE, "snn_step_route called before snn_deliver");
  const bool fused = mode != SNN_ROUTE_FLAT && fused_route_ok(h->kp);
  HIP_TRY(launch_update(h->kp, h->stream, nullptr, fused));
  HIP_TRY(launch_route(h->kp, mode, h->stream, nullptr, fused, true));
  h->route_mode = mode;
  h->expand_deferred = true;
  h->phase = 2;
  h->routed_t = h->t_host + 1;
  return SNN_OK;
}

// One whole step in route mode `mode`: two-level routing inside the update
// kernel where the node count allows, mask expansion inside the staging.
static hipError_t launch_step(const KParams& kp, int mode, hipStream_t s, hipEvent_t* marks) {
  const bool fused = mode != SNN_ROUTE_FLAT && fused_route_ok(kp);
  hipError_t e = launch_update(kp, s, marks, fused);
  if (e == hipSuccess) e = launch_route(kp, mode, s, marks, fused, true);
  if (e == hipSuccess) e = launch_deliver(kp, mode, s, marks, true);
  return e;
}

// The same step with the neuron update (and its routing) launched once per
// partition, over that partition's neurons [start[p], start[p+1]) only: the
// launches of a step append their fired ids in partition order, and the last
// one advances the step.  The receive side is one launch set as above.
static hipError_t launch_step_partitioned(const KParams& kp, int mode, hipStream_t s,
                                          const std::vector<uint32_t>& start) {
  const bool fused = mode != SNN_ROUTE_FLAT && fused_route_ok(kp);
  const uint32_t P = static_cast<uint32_t>(start.size()) - 1;
  uint32_t last = P;
  for (uint32_t p = 0; p < P; ++p)
    if (start[p + 1] > start[p]) last = p;
  hipError_t e = hipSuccess;
  for (uint32_t p = 0; p < P && e == hipSuccess; ++p) {
    if (start[p + 1] == start[p]) continue;
    KParams q = kp;
    q.lo = start[p];
    q.hi = start[p + 1];
    q.tile0 = q.lo / kp.tile;
    q.tile_end = (q.hi - 1) / kp.tile + 1;
    q.step_ends = p == last ? 1u : 0u;
    e = launch_update(q, s, nullptr, fused);
  }
  if (e == hipSuccess) e = launch_route(kp, mode, s, nullptr, fused, true);
  if (e == hipSuccess) e = launch_deliver(kp, mode, s, nullptr, true);
  return e;
}

static hipError_t launch_step_as(snn_handle h, int layout, int mode) {
  return layout ? launch_step_partitioned(h->kp, mode, h->stream, h->part_start)
                : launch_step(h->kp, mode, h->stream, nullptr);
}

snn_status snn_deliver(snn_handle h) {
  if (!h) return fail(SNN_ERR_INVALID_ARG, "handle is NULL");
  if (h->phase != 2) return fail(SNN_ERR_BAD_STATE, "snn_deliver must follow snn_route");
  if (h->expand_deferred && handoff_used(h, h->route_mode) && handoff_tag_repeats(h)) {
    KParams q = h->kp;
    q.recv_merged = 0;
    HIP_TRY(launch_deliver(q, h->route_mode, h->stream, nullptr, true));
  } else {
    HIP_TRY(launch_deliver(h->kp, h->route_mode, h->stream, nullptr, h->expand_deferred));
    if (h->expand_deferred && handoff_used(h, h->route_mode)) h->handoff_t = h->t_host + 1;
  }
  h->expand_deferred = false;
  h->phase = 0;
  h->t_host += 1;
  return SNN_OK;
}

// Captures n steps of the given layout and mode into one executable graph.
static snn_status capture_steps(snn_handle h, int layout, int mode, uint32_t steps,
                                hipGraphExec_t* out) {
  hipGraph_t g = nullptr;
  HIP_TRY(hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e = hipSuccess;
  for (uint32_t i = 0; i < steps && e == hipSuccess; ++i) e = launch_step_as(h, layout, mode);
  hipError_t ec = hipStreamEndCapture(h->stream, &g);
  if (e != hipSuccess || ec != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return fail(SNN_ERR_HIP, "graph capture failed: %s",
                hipGetErrorString(e != hipSuccess ? e : ec));
  }
  hipError_t ei = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (ei != hipSuccess) {
    *out = nullptr;
    return fail(SNN_ERR_HIP, "hipGraphInstantiate: %s", hipGetErrorString(ei));
  }
  return SNN_OK;
}

// Every captured graph holds the kernel parameters of its capture: dropped
// when they change.
static void drop_graphs(snn_handle h) {
  for (auto& gl : h->graph)
    for (auto& gm : gl)
      for (auto& g : gm)
        if (g) {
          (void)hipGraphExecDestroy(g);
          g = nullptr;
        }
  if (h->whole) (void)hipGraphExecDestroy(h->whole);
  h->whole = nullptr;
}

static snn_status run_steps(snn_handle h, uint32_t n_steps, int mode, int use_graph, int layout) {
  if (mode < SNN_ROUTE_TWO_LEVEL || mode > SNN_ROUTE_BOTH)
    return fail(SNN_ERR_INVALID_ARG, "route mode %d", mode);
  if (use_graph < 0 || use_graph > 2) return fail(SNN_ERR_INVALID_ARG, "use_graph %d", use_graph);
  if (h->phase != 0) return fail(SNN_ERR_BAD_STATE, "snn_run called in the middle of a step");
  if (use_graph && h->is_static)
    return fail(SNN_ERR_UNSUPPORTED, "snn_run: a handle from snn_create_static runs without "
                "HIP graphs (instantiating one allocates)");
  if (n_steps == 0) return SNN_OK;
  const bool handoff = handoff_used(h, mode);
  if (handoff && handoff_tag_repeats(h)) {
    KParams q = h->kp;
    q.recv_merged = 0;
    HIP_TRY(layout ? launch_step_partitioned(q, mode, h->stream, h->part_start)
                   : launch_step(q, mode, h->stream, nullptr));
    h->route_mode = mode;
    h->t_host += 1;
    h->routed_t = h->t_host;
    if (--n_steps == 0) return SNN_OK;
  }
  if (!use_graph) {
    for (uint32_t i = 0; i < n_steps; ++i) HIP_TRY(launch_step_as(h, layout, mode));
  } else if (use_graph == 2) {
    const uint32_t key[3] = {n_steps, uint32_t(mode), uint32_t(layout)};
    if (h->whole && std::memcmp(key, h->whole_key, sizeof(key)) != 0) {
      (void)hipGraphExecDestroy(h->whole);
      h->whole = nullptr;
    }
    if (!h->whole) {
      snn_status st = capture_steps(h, layout, mode, n_steps, &h->whole);
      if (st != SNN_OK) return st;
      std::memcpy(h->whole_key, key, sizeof(key));
    }
    HIP_TRY(hipGraphLaunch(h->whole, h->stream));
  } else {
    const uint32_t n_long = n_steps / GRAPH_STEPS, n_short = n_steps % GRAPH_STEPS;
    for (int which = 1; which >= 0; --which) {
      const uint32_t reps = which ? n_long : n_short;
      if (!reps) continue;
      hipGraphExec_t& g = h->graph[layout][mode][which];
      if (!g) {
        snn_status st = capture_steps(h, layout, mode, which ? GRAPH_STEPS : 1u, &g);
        if (st != SNN_OK) return st;
      }
      for (uint32_t i = 0; i < reps; ++i) HIP_TRY(hipGraphLaunch(g, h->stream));
    }
  }
  h->route_mode = mode;
  h->t_host += n_steps;
  h->routed_t = h->t_host;
  if (handoff) h->handoff_t = h->t_host;
  return SNN_OK;
}

snn_status snn_run(snn_handle h, uint32_t n_steps, int mode, int use_graph) {
  if (!h) return fail(SNN_ERR_INVALID_ARG, "handle is NULL");
  return run_steps(h, n_steps, mode, use_graph, 0);
}

snn_status snn_run_partitioned(snn_handle h, uint32_t n_steps, int mode, int use_graph,
                               const uint32_t* part_start) {
  if (!h || !part_start) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  if (h->is_static)
    return fail(SNN_ERR_UNSUPPORTED, "snn_run_partitioned: not for a handle from "
                "snn_create_static (it keeps a host copy of the partition starts)");
  const uint32_t P = h->kp.P;
  if (part_start[0] != 0 || part_start[P] != h->kp.N)
    return fail(SNN_ERR_INVALID_ARG, "part_start must run from 0 to n_neurons (%u)", h->kp.N);
  for (uint32_t p = 0; p < P; ++p)
    if (part_start[p + 1] < part_start[p])
      return fail(SNN_ERR_INVALID_ARG, "part_start decreases at partition %u", p);
  if (h->part_start.size() != P + 1 ||
      !std::equal(h->part_start.begin(), h->part_start.end(), part_start)) {
    for (auto& gm : h->graph[1])
      for (auto& g : gm)
        if (g) {
          (void)hipGraphExecDestroy(g);
          g = nullptr;
        }
    if (h->whole && h->whole_key[2] == 1) {
      (void)hipGraphExecDestroy(h->whole);
      h->whole = nullptr;
    }
    h->part_start.assign(part_start, part_start + P + 1);
  }
  return run_steps(h, n_steps, mode, use_graph, 1);
}

snn_status snn_set_tuning(snn_handle h, const snn_tuning* t) {
  if (!h || !t) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  if (h->phase != 0) return fail(SNN_ERR_BAD_STATE, "snn_set_tuning called in the middle of a step");
  if (t->update_blocks > h->kp.n_tiles)
    return fail(SNN_ERR_INVALID_ARG, "update_blocks %u > %u tiles", t->update_blocks, h->kp.n_tiles);
  if (t->recv_split > STAGE_BLOCKS)
    return fail(SNN_ERR_INVALID_ARG, "recv_split %u > %u", t->recv_split, STAGE_BLOCKS);
  if (t->recv_merged > 1) return fail(SNN_ERR_INVALID_ARG, "recv_merged %u", t->recv_merged);
  if (h->kp.update_blocks != t->update_blocks || h->kp.recv_split != t->recv_split ||
      h->kp.recv_merged != t->recv_merged) {
    HIP_TRY(hipStreamSynchronize(h->stream));
    drop_graphs(h);
    h->kp.update_blocks = t->update_blocks;
    h->kp.recv_split = t->recv_split;
    h->kp.recv_merged = t->recv_merged;
  }
  return SNN_OK;
}

snn_status snn_get_tuning(snn_handle h, snn_tuning* t) {
  if (!h || !t) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  t->update_blocks = h->kp.update_blocks;
  t->recv_split = h->kp.recv_split;
  t->recv_merged = h->kp.recv_merged;
  return SNN_OK;
}

static snn_status sync_and_check(snn_handle h, DevState* out);

snn_status snn_kernel_times(snn_handle h, uint32_t n_steps, int mode, float* avg_ms) {
  if (!h || !avg_ms) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  if (mode < SNN_ROUTE_TWO_LEVEL || mode > SNN_ROUTE_BOTH)
    return fail(SNN_ERR_INVALID_ARG, "route mode %d", mode);
  if (h->phase != 0) return fail(SNN_ERR_BAD_STATE, "snn_kernel_times called in the middle of a step");
  // Every step gets its own events and nothing synchronises until the end:
  // the launches queue up behind each other as in a normal run, so no start
  // event fires on an idle queue ahead of its kernel.
  const bool fused = mode != SNN_ROUTE_FLAT && fused_route_ok(h->kp);
  // expansion and staging of a two-level step share the receive-side launch,
  // and so does the remote delivery when that side is one launch
  const bool launched[SNN_NKERNEL] = {true,
                                      mode != SNN_ROUTE_FLAT && !fused,
                                      false,
                                      mode != SNN_ROUTE_TWO_LEVEL,
                                      true,
                                      mode == SNN_ROUTE_FLAT || !h->kp.recv_merged};
  std::vector<hipEvent_t> marks(size_t(2) * SNN_NKERNEL * n_steps, nullptr);
  snn_status st = SNN_OK;
  for (auto& e : marks) {
    hipError_t r = hipEventCreate(&e);
    if (r != hipSuccess) {
      st = fail(SNN_ERR_HIP, "hipEventCreate: %s", hipGetErrorString(r));
      break;
    }
  }
  double total[SNN_NKERNEL] = {};
  const bool handoff = handoff_used(h, mode);
  for (uint32_t i = 0; i < n_steps && st == SNN_OK; ++i) {
    hipEvent_t* m = marks.data() + size_t(2) * SNN_NKERNEL * i;
    KParams q = h->kp;
    if (handoff && handoff_tag_repeats(h)) q.recv_merged = 0;   // see handoff_tag_repeats
    else if (handoff) h->handoff_t = h->t_host + 1;
    hipError_t r = launch_step(q, mode, h->stream, m);
    if (r != hipSuccess) st = fail(SNN_ERR_HIP, "timed step: %s", hipGetErrorString(r));
    h->t_host += 1;
    h->route_mode = mode;
    h->routed_t = h->t_host;
  }
  if (st == SNN_OK) {
    hipError_t r = hipStreamSynchronize(h->stream);
    if (r != hipSuccess) st = fail(SNN_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(r));
  }
  for (uint32_t i = 0; i < n_steps && st == SNN_OK; ++i)
    for (int k = 0; k < SNN_NKERNEL && st == SNN_OK; ++k) {
      if (!launched[k]) continue;
      const hipEvent_t* m = marks.data() + size_t(2) * SNN_NKERNEL * i;
      float ms = 0.f;
      hipError_t r = hipEventElapsedTime(&ms, m[2 * k], m[2 * k + 1]);
      if (r != hipSuccess) st = fail(SNN_ERR_HIP, "hipEventElapsedTime: %s", hipGetErrorString(r));
      total[k] += ms;
    }
  for (auto& e : marks)
    if (e) (void)hipEventDestroy(e);
  if (st != SNN_OK) return st;
  for (int k = 0; k < SNN_NKERNEL; ++k)
    avg_ms[k] = launched[k] && n_steps ? static_cast<float>(total[k] / n_steps) : 0.f;
  return sync_and_check(h, nullptr);
}

snn_status snn_flush(snn_handle h) {
  if (!h) return fail(SNN_ERR_INVALID_ARG, "handle is NULL");
  if (h->phase != 0) return fail(SNN_ERR_BAD_STATE, "snn_flush called in the middle of a step");
  HIP_TRY(launch_flush(h->kp, h->stream));
  return SNN_OK;
}

static snn_status sync_and_check(snn_handle h, DevState* out) {
  HIP_TRY(hipStreamSynchronize(h->stream));
  DevState st;
  HIP_TRY(hipMemcpy(&st, h->kp.st, sizeof(st), hipMemcpyDeviceToHost));
  if (out) *out = st;
  if (st.error & ERR_ROUTE)
    return fail(SNN_ERR_HIP, "receive entry without a matching destination partition");
  if (st.error & ERR_TIMEOUT)
    return fail(SNN_ERR_HIP, "a wait between blocks of one launch timed out");
  if (st.error & ERR_XCD)
    return fail(SNN_ERR_UNSUPPORTED, "the one-launch receive side found a queue staged on "
                "another XCD than the block that bins it (workgroups are not dealt out to the "
                "XCDs in turn on this device); use the two-launch receive side "
                "(recv_merged = 0)");
  if (st.error)
    return fail(SNN_ERR_CAPACITY, "device capacity overflow (bits 0x%x: 1 bucket, 2 receive "
                "list, 4 flat list, 8 spike log)", st.error);
  return SNN_OK;
}

snn_status snn_sync(snn_handle h) {
  if (!h) return fail(SNN_ERR_INVALID_ARG, "handle is NULL");
  return sync_and_check(h, nullptr);
}

uint64_t snn_time(snn_handle h) { return h ? h->t_host : 0; }

snn_status snn_bin_geometry(const snn_params* params, uint32_t* tile_neurons,
                            uint32_t* deliver_blocks, uint32_t* stage_blocks) {
  if (!params) return fail(SNN_ERR_INVALID_ARG, "params is NULL");
  snn_status st = check_tile(params);
  if (st != SNN_OK) return st;
  if (tile_neurons) *tile_neurons = tile_size(params->n_neurons, params->tile_neurons);
  if (deliver_blocks) *deliver_blocks = DELIVER_BLOCKS;
  if (stage_blocks) *stage_blocks = STAGE_BLOCKS;
  return SNN_OK;
}

snn_status snn_ring_events(snn_handle h, uint64_t* n) {
  if (!h || !n) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  DevState st;
  snn_status s = sync_and_check(h, &st);
  *n = st.ring_events;
  return s;
}

snn_status snn_read_counters(snn_handle h, uint64_t first_step, uint32_t n_steps, uint64_t* out) {
  if (!h || (!out && n_steps)) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  const uint64_t L = h->prm.log_steps;
  if (first_step + n_steps > h->t_host || first_step + L < h->t_host)
    return fail(SNN_ERR_INVALID_ARG, "steps [%llu, %llu) not among the last %llu of %llu",
                (unsigned long long)first_step, (unsigned long long)(first_step + n_steps),
                (unsigned long long)L, (unsigned long long)h->t_host);
  if (n_steps > L) return fail(SNN_ERR_INVALID_ARG, "n_steps exceeds log_steps");
  snn_status s = sync_and_check(h, nullptr);
  if (s != SNN_OK && s != SNN_ERR_CAPACITY) return s;
  std::vector<uint64_t> all(STAT_ROW_WORDS * (L + 1));
  HIP_TRY(hipMemcpy(all.data(), h->kp.stats, all.size() * 8, hipMemcpyDeviceToHost));
  for (uint32_t i = 0; i < n_steps; ++i) {
    const uint64_t* row = all.data() + ((first_step + i) % (L + 1)) * STAT_ROW_WORDS;
    for (uint32_t k = 0; k < SNN_NSTAT; ++k) {
      uint64_t v = 0;
      for (uint32_t c = 0; c < STAT_LANES; ++c) v += row[c * STAT_LANE_WORDS + k];
      out[uint64_t(i) * SNN_NSTAT + k] = v;
    }
  }
  return s;
}

snn_status snn_read_spikes(snn_handle h, uint64_t first_step, uint32_t n_steps, int32_t* ids,
                           uint64_t cap, uint32_t* per_step_counts, uint64_t* n_ids) {
  if (!h || !n_ids) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  *n_ids = 0;
  const uint64_t L = h->prm.log_steps;
  if (first_step + n_steps > h->t_host || first_step + L < h->t_host || n_steps > L)
    return fail(SNN_ERR_INVALID_ARG, "steps [%llu, %llu) not among the last %llu of %llu",
                (unsigned long long)first_step, (unsigned long long)(first_step + n_steps),
                (unsigned long long)L, (unsigned long long)h->t_host);
  HIP_TRY(hipStreamSynchronize(h->stream));
  DevState st;
  HIP_TRY(hipMemcpy(&st, h->kp.st, sizeof(st), hipMemcpyDeviceToHost));
  std::vector<uint64_t> stats(STAT_ROW_WORDS * (L + 1)), offs(L);
  HIP_TRY(hipMemcpy(stats.data(), h->kp.stats, stats.size() * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(offs.data(), h->kp.log_off, offs.size() * 8, hipMemcpyDeviceToHost));
  const uint64_t logcap = h->prm.log_cap;
  uint64_t total = 0;
  for (uint32_t i = 0; i < n_steps; ++i) {
    const uint64_t r = (first_step + i) % L;
    const uint64_t cnt = stats[((first_step + i) % (L + 1)) * STAT_ROW_WORDS + SNN_STAT_SPIKES];
    if (per_step_counts) per_step_counts[i] = uint32_t(cnt);
    // still in the log ring?
    if (cnt && (logcap == 0 || st.log_total - offs[r] > logcap))
      return fail(SNN_ERR_CAPACITY, "spikes of step %llu are no longer in the spike log",
                  (unsigned long long)(first_step + i));
    total += cnt;
  }
  *n_ids = total;
  if (!ids) return SNN_OK;
  if (total > cap) return fail(SNN_ERR_CAPACITY, "%llu ids do not fit cap %llu",
                               (unsigned long long)total, (unsigned long long)cap);
  uint64_t at = 0;
  for (uint32_t i = 0; i < n_steps; ++i) {
    const uint64_t r = (first_step + i) % L;
    uint64_t cnt = stats[((first_step + i) % (L + 1)) * STAT_ROW_WORDS + SNN_STAT_SPIKES];
    if (!cnt) continue;
    uint64_t pos = offs[r] % logcap;
    while (cnt) {
      const uint64_t piece = std::min(cnt, logcap - pos);
      HIP_TRY(hipMemcpy(ids + at, h->kp.log + pos, piece * 4, hipMemcpyDeviceToHost));
      at += piece;
      cnt -= piece;
      pos = 0;
    }
  }
  return SNN_OK;
}

snn_status snn_read_routes(snn_handle h, int which, uint64_t* sizes, void* entries, uint64_t cap,
                           uint64_t* n_entries) {
  if (!h || !sizes || !n_entries) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  if (which < 0 || which > 2) return fail(SNN_ERR_INVALID_ARG, "which=%d", which);
  if (!h->routed_t) return fail(SNN_ERR_BAD_STATE, "no step has been routed yet");
  const int mode = h->route_mode;
  if ((which == 0 && mode == SNN_ROUTE_TWO_LEVEL) || (which != 0 && mode == SNN_ROUTE_FLAT))
    return fail(SNN_ERR_BAD_STATE, "the last step was not routed in a mode that fills these buffers");
  if (which == 1 && h->expand_deferred)
    return fail(SNN_ERR_BAD_STATE, "after snn_step_route the receive lists are filled by snn_deliver");
  DevState dst;
  snn_status s = sync_and_check(h, &dst);
  if (s != SNN_OK) return s;
  const uint32_t nl = which == 2 ? h->kp.n_nodes : h->kp.P;
  std::vector<uint32_t> cnt(uint64_t(nl) * CNT_STRIDE);
  std::vector<uint64_t> off(nl + 1);
  const uint32_t* cnt_dev = which == 0   ? h->kp.flat_cnt
                            : which == 1 ? h->kp.recv_cnt
                                         : h->kp.bucket_cnt + uint64_t(dst.cur_par) * nl * CNT_STRIDE;
  const uint64_t* off_dev = which == 2 ? h->kp.bucket_off : h->kp.recv_off;
  HIP_TRY(hipMemcpy(cnt.data(), cnt_dev, cnt.size() * 4, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(off.data(), off_dev, (nl + 1) * 8, hipMemcpyDeviceToHost));
  uint64_t total = 0;
  for (uint32_t i = 0; i < nl; ++i) {
    sizes[i] = cnt[uint64_t(i) * CNT_STRIDE];
    total += sizes[i];
  }
  *n_entries = total;
  if (!entries) return SNN_OK;
  if (total > cap) return fail(SNN_ERR_CAPACITY, "%llu entries do not fit cap %llu",
                               (unsigned long long)total, (unsigned long long)cap);
  const char* base = which == 0 ? reinterpret_cast<const char*>(h->kp.flat)
                     : which == 1 ? reinterpret_cast<const char*>(h->kp.recv)
                                  : reinterpret_cast<const char*>(h->kp.bucket);
  uint64_t at = 0;
  for (uint32_t i = 0; i < nl; ++i) {
    if (!sizes[i]) continue;
    const uint64_t w = which == 2 ? 16 : 8;   // a message is two words
    HIP_TRY(hipMemcpyAsync(static_cast<char*>(entries) + at * w, base + off[i] * w, sizes[i] * w,
                           hipMemcpyDeviceToHost, h->stream));
    at += sizes[i];
  }
  HIP_TRY(hipStreamSynchronize(h->stream));
  return SNN_OK;
}

snn_status snn_destroy(snn_handle h) {
  if (!h) return SNN_OK;
  snn_status s = SNN_OK;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) s = fail(SNN_ERR_HIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
  if (h->is_static) return s;   // static storage: never freed (a newer static
                                // handle of the device may already use it)
  drop_graphs(h);
  delete h;
  return s;
}

}  // extern "C"
