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
  ERR_ROUTE = 16u,   // a receive entry names a partition its source does not reach
  ERR_TIMEOUT = 32u, // a wait between blocks of one launch gave up (a block it waited for
                     // never arrived)
  ERR_XCD = 64u      // a queue of the one-launch receive side was staged on another XCD
                     // than the block that bins it (the hand-off needs a shared L2)
};

// Words of the in-launch synchronisation area (KParams::sync), each on a
// 64-byte line of its own; they hold tagged values, so nothing clears them.
enum : uint32_t {
  SYNC_STRIDE = 16,   // words per line
  SYNC_WORDS = 256 * SYNC_STRIDE    // word SYNC_STRIDE * b: staging block b's flag
};

// Device-resident step state.  Every step-dependent value lives here so that
// a captured step replays unchanged.
// Residues of t are kept alongside it (advanced by the update kernel's last
// block) so kernels never divide 64-bit values.
struct DevState {
  uint64_t t;          // step the next update kernel runs
  uint64_t log_total;  // ids appended to the spike log so far
  uint32_t n_fired;    // spikes of the step in flight (t - 1 after the update)
  uint32_t error;      // sticky ERR_* bits
  uint64_t ring_events;  // events that went to the dense ring (bin or staging full)
  uint32_t slot;       // t mod D
  uint32_t row;        // t mod log_steps
  uint32_t phase;      // t mod raster_period
  uint32_t tag;        // look-back tag of step t, minus 1, in [0, 2^30 - 1)
  uint32_t cur_slot;   // slot of the step in flight
  uint32_t cur_row;    // row of the step in flight
  uint64_t log_head;   // log_total mod log_cap
  uint32_t cur_par;    // parity (t mod 2) of the step in flight: its bucket counter set
  uint32_t srow;       // t mod (log_steps + 1): counter row of step t
  uint32_t cur_srow;   // counter row of the step in flight
  uint32_t part_base;  // fired ids of the step so far, while its update runs as one launch
                       // per partition (0 between steps)
};

// Stream ids of the counter-based generator.
enum : uint32_t { STREAM_POISSON = 1u, STREAM_RASTER = 2u };

// Geometry.  Neurons are grouped in tiles of T neurons (KParams::tile, a
// multiple of TILE_ALIGN up to TILE_MAX, fixed per network): the update
// kernel runs one block per tile and accumulates the tile's arriving input
// in LDS; synaptic events are binned per (ring slot, tile).  The default T
// is the largest (TILE_MAX), unless that leaves fewer than TILE_MIN_COUNT
// tiles (two update blocks per CU of a 256-CU part); then the neurons are
// spread over TILE_MIN_COUNT tiles, down to TILE_MIN_DEFAULT neurons each.
// Larger tiles mean fewer sub-bins, so longer runs per sub-bin in the
// delivery; more tiles keep every CU busy where the network is small.
constexpr uint32_t TILE_MAX = 8192;
constexpr uint32_t TILE_ALIGN = 64;
constexpr uint32_t TILE_MIN_DEFAULT = 2048;
constexpr uint32_t TILE_MIN_COUNT = 2 * 256;
constexpr int UPDATE_THREADS = 512;
constexpr int UPDATE_NPT = TILE_MAX / UPDATE_THREADS;   // 16 neurons per thread at most
constexpr int ROUTE_THREADS = 256;
constexpr int DELIVER_THREADS = 512;
constexpr uint32_t CNT_STRIDE = 16;                 // counters padded to 64 bytes
constexpr uint32_t ROUTE_STAGE = 2048;              // pairs per routing window
constexpr uint32_t ROUTE_BLOCKS = 256;              // two-level routing blocks
constexpr uint32_t ROUTE_MAX_NODES_LDS = 4096;      // more nodes: unstaged routing
constexpr uint32_t DELIVER_BLOCKS = 32;             // deliver blocks per delay
// XCDs of the chip (each with its own L2): workgroup b of a launch runs on XCD
// (b + c) mod N_XCD for a c fixed per launch, so blocks whose indices differ
// by a multiple of N_XCD share an XCD.  The one-launch receive side relies on
// that (and checks it at run time).
constexpr uint32_t N_XCD = 8;
constexpr uint32_t STAGE_BLOCKS = 256;              // receive-side blocks (one queue each)
constexpr uint32_t STAGE_PARTS = 256;               // partitions per receive-side block, at most
static_assert(STAGE_PARTS * STAGE_BLOCKS >= SNN_MAX_PARTITIONS, "receive blocks must cover P");
static_assert(STAGE_BLOCKS % DELIVER_BLOCKS == 0, "deliver blocks split the queues evenly");
constexpr int RECV_THREADS = 512;
constexpr uint32_t RECV_PER_THREAD = 4;                         // entries per thread per batch
constexpr uint32_t RECV_BATCH = RECV_THREADS * RECV_PER_THREAD; // entries per batch
static_assert(STAGE_PARTS <= RECV_THREADS, "one partition count per thread");
constexpr uint32_t EXPAND_BUF = 2048;               // receive entries buffered per staging pass
constexpr uint32_t EXPAND_PER_THREAD = 4;           // messages per thread per expansion round
static_assert(EXPAND_BUF >= SNN_MAX_GPUS_PER_NODE, "one message's entries fit the buffer");

// Per-step counters: each row (step mod (log_steps + 1); the spare row is the
// next step's, cleared by the update kernel ahead of its use) holds STAT_LANES copies of
// the SNN_NSTAT counters, one 128-byte line each.  A block adds into copy
// (block index mod STAT_LANES), so the per-block atomics of a kernel spread
// over STAT_LANES lines instead of queueing on one; the host sums the copies.
// The spike count is written once, into copy 0.
constexpr uint32_t STAT_LANES = 16;
constexpr uint32_t STAT_LANE_WORDS = 16;
constexpr uint32_t STAT_ROW_WORDS = STAT_LANES * STAT_LANE_WORDS;
static_assert(SNN_NSTAT <= STAT_LANE_WORDS, "a copy of the counters fits its line");

// Poisson inversion lookup: entry b covers draws r in [b << POIS_LUT_SHIFT,
// (b + 1) << POIS_LUT_SHIFT).  k = #{j : thr[j] <= r} is the entry itself
// when no threshold lies inside that range (entry < 16); with exactly one,
// thr[j] with j = entry - 16, it is j + (r >= thr[j]); POIS_LUT_SLOW marks
// ranges holding several thresholds, where the kernel counts all 15.
constexpr int POIS_LUT_SHIFT = 19;
constexpr uint32_t POIS_LUT_SIZE = 1u << (32 - POIS_LUT_SHIFT);   // 8192 one-byte entries
constexpr uint8_t POIS_LUT_SLOW = 255;

// Receive-list entries: source id in the low ENTRY_SRC_BITS bits (ids are
// below 2^27), the (source, partition) pair index above.
constexpr int ENTRY_SRC_BITS = 27;
constexpr uint64_t ENTRY_SRC_MASK = (uint64_t(1) << ENTRY_SRC_BITS) - 1;

// Synaptic input is summed in fixed point: each binned event carries its
// weight rounded to a multiple of 2^-F (int32), the update adds them exactly
// with 32-bit LDS integer atomics (about ten times faster than float ones on
// gfx950) and rounds the sum once to binary32.  F comes from the bound on a
// neuron's input in one step (snn_params.input_bound), so the sum cannot
// overflow; sums of weights that are multiples of 2^-F are exact.

// A binned synaptic event: target index (inside its tile in the bins, global
// in the receive queues) and quantized weight.
struct Event {
  uint32_t tgt;
  int32_t wq;   // weight in units of 2^-F
};

// Everything a kernel needs, passed by value.
struct KParams {
  // model
  uint32_t N, P, G, D, n_nodes, n_tiles;
  uint32_t g_magic;          // ceil(2^32 / G) for G >= 2: node of a partition by one multiply
  uint32_t tile;             // neurons per tile, T
  uint32_t tile_magic, tile_shift;   // x / T = umulhi(x, tile_magic) >> tile_shift, x < 2^27
  uint32_t n_ref;
  uint64_t ring_stride;
  float alpha, theta, u_reset, w_ext;
  uint32_t thr[15];
  const uint8_t* pois_lut;   // [POIS_LUT_SIZE] (workspace)
  uint32_t seed_lo, seed_hi;
  uint32_t forced, raster_on_thr, raster_off_thr, raster_period, raster_on;
  uint32_t bf16;
  uint32_t log_steps;
  uint64_t log_cap;
  uint64_t bin_cap;
  uint64_t stage_cap;
  uint32_t recv_split;   // most receive-side blocks sharing one node's bucket (0 = as many
                         // as the blocks allow); tunable per shape
  // what one update launch covers: tiles [tile0, tile_end), neurons [lo, hi);
  // step_ends: the step's last update launch (advances the step state).  A
  // whole-step launch has tile0 = 0, tile_end = n_tiles, lo = 0, hi = N.
  uint32_t tile0, tile_end, lo, hi, step_ends;
  uint32_t update_blocks;   // grid of a whole-step update launch (0: one block per tile;
                            // fewer: persistent blocks taking tiles in ticket order)
  uint32_t recv_merged;     // receive side of a whole step in one launch (1) or two (0)
  float wq_scale;      // 2^F: weight -> fixed point
  double wq_inv;       // 2^-F
  // network (caller-owned device memory)
  const int64_t* row_ptr;
  const uint32_t* n_local;
  const uint16_t* delay_off;   // [N][D] start of each delay's run in the local segment
  const uint32_t* tgt_delay;
  const void* weight;
  const int64_t* vp_ptr;
  const uint16_t* vp_part;
  const uint64_t* vp_rec;     // [2 * pairs] receive records (start | len << 40, first synapse)
  const int32_t* part;
  const uint64_t* bucket_off;
  const uint64_t* recv_off;
  uint64_t n_pairs;           // vp_ptr[N]: destination pairs (bounds checks)
  uint64_t nnz;               // row_ptr[N]: synapses (bounds checks)
  float* u;
  uint8_t* ref;
  float* ring;               // read-back view of the pending input (snn_flush)
  // workspace
  int32_t* ovf;         // [D][ring_stride] overflow ring: fixed-point input of events that
                        // did not fit their bin or staging queue
  DevState* st;
  uint64_t* lookback;   // [n_tiles] decoupled look-back words
  uint32_t* tickets;    // [2] tiles handed out by a persistent update, by step parity
  uint32_t* sync;       // [SYNC_WORDS] in-launch arrival counters
  uint32_t* fired;      // [N] ascending fired ids of the step in flight
  uint32_t* bucket_cnt; // [2][n_nodes * CNT_STRIDE] two sets, by step parity
  uint64_t* bucket;     // [2 * bucket_total] messages: source | pair index of the
                        // node's first destination << 32, then the partition mask
  uint32_t* recv_cnt;   // [P * CNT_STRIDE] expanded lists
  uint64_t* recv;       // [recv_total]
  uint32_t* flat_cnt;   // [P * CNT_STRIDE]
  uint64_t* flat;       // [recv_total]
  uint32_t* stage_cnt;  // [max_delay * CNT_STRIDE] remote events staged per delay
  Event* stage;         // [max_delay][stage_cap] (global target ids)
  uint32_t* bin_cnt;    // [D * n_tiles * max_delay * DELIVER_BLOCKS], see subbin()
  uint32_t* dirty;      // [D * n_tiles] ring tile holds events
  Event* bins;          // [D][n_tiles][bin_cap]
  uint64_t* stats;      // [log_steps + 1][STAT_LANES][STAT_LANE_WORDS]
  uint64_t* log_off;    // [log_steps] first log position of each step
  uint32_t* log;        // [log_cap] spike-log ring
};

// Launchers (snn_kernels.hip); all enqueue on `s` and return the launch error.
// With non-null marks, events marks[2k], marks[2k + 1] are recorded around
// each launch of kernel kind k (SNN_KERNEL_*).
// Tile size for n neurons and a requested size (0: the default rule), and
// the multiplier and shift that divide by it.
uint32_t tile_size(uint32_t n, uint32_t requested);
void tile_divider(uint32_t t, uint32_t* magic, uint32_t* shift);
hipError_t prepare_kernels(KParams& p);   // LDS limits of the kernels, once per handle
// With route, the update kernel also routes the step two-level where the node
// count allows (fused_route_ok); launch_route is then told so (routed) and
// launches only what remains (expansion, flat lists).
bool fused_route_ok(const KParams& p);
hipError_t launch_update(const KParams& p, hipStream_t s, hipEvent_t* marks = nullptr,
                         bool route = false);
// With defer_expand, launch_route leaves the mask expansion to launch_deliver
// (fused_expand), which then expands and stages in one kernel.
hipError_t launch_route(const KParams& p, int mode, hipStream_t s, hipEvent_t* marks = nullptr,
                        bool routed = false, bool defer_expand = false);
hipError_t launch_deliver(const KParams& p, int mode, hipStream_t s, hipEvent_t* marks = nullptr,
                          bool fused_expand = false);
hipError_t launch_flush(const KParams& p, hipStream_t s);
// Set-up without memset or host copies: zeroes bytes (a multiple of 4) at
// dst; builds the Poisson lookup from p.thr into lut.
hipError_t launch_zero(void* dst, uint64_t bytes, hipStream_t s);
hipError_t launch_pois_lut(const KParams& p, uint8_t* lut, hipStream_t s);

}  // namespace snn
