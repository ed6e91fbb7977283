// snn_kernels.hip — the per-step kernels for gfx950 (wave64, CDNA4).
//
// The work of a step, as device functions shared by the kernels:
//   k_update       one block per tile of T neurons: sums the tile's arriving
//                  synaptic events into LDS from its bins, runs the LIF update
//                  and threshold, compacts fired ids in ascending order (wave
//                  ballots, block scan, decoupled look-back across tiles)
//   route_batch    two-level routing: one (source, node mask) message per
//                  destination node into per-node buckets (Sec. IV-B)
//   expand_stage_block / k_expand
//                  mask expansion into per-partition receive lists (the
//                  bridge's forwarding)
//   stage_batch    receive side: each entry's synapses for its partition,
//                  staged per delay in per-block queues
//   deliver_block  per delay: the own-partition synapses of fired sources and
//                  the staged remote ones, counting-sorted by tile in LDS and
//                  written as runs into per-(slot, tile, delay, block) bins
//   k_route_flat   flat routing: one receive entry per destination partition
//
// A whole step is two or three launches: k_update<true> (update, compaction
// and the tile's own two-level routing, which overlaps the look-back), then
// the receive side in one of two forms (snn_tuning.recv_merged, one launch
// by default):
//   k_recv_local + k_deliver_remote: expansion and staging beside the
//     own-partition delivery, then the staged remote synapses in a launch of
//     their own, appended after the counts the local part published;
//   k_recv_deliver: the same in one launch, the delivery blocks waiting for
//     the staging blocks and then binning the staged remote synapses too.
//     Every queue is written and read by blocks on the same XCD (workgroups
//     are dealt out to the XCDs in turn, and the queue of staging block b is
//     binned by delivery blocks whose index is b mod 8 apart from it by a
//     multiple of 8), so the queues pass through that XCD's L2 with plain
//     stores and loads: no write-back of the (non-coherent, per-XCD) L2,
//     which a device-scope release per block would cost, and no
//     write-through stores.  Each staging block publishes the XCD it ran on
//     with its flag, and a delivery block flags ERR_XCD for a queue staged
//     on another XCD than its own.
// The step-by-step entry points use one kernel per job instead
// (k_update<false>, k_route_two_level, k_expand, k_recv_stage, k_deliver).
//
// Global atomics run at roughly 20 G/s on random addresses and serialise on
// hot counters, so every scatter goes through LDS first: reservations are one
// atomic per round and counter (routing), or none at all (the bins are private
// per writer and written once per ring cycle).  The dense delay ring is only a
// fallback for events that do not fit their bin; its tiles are read when
// flagged.  The work is sparse gather/scatter: no dense contraction, no MFMA.
// Compiled with -ffp-contract=off: the membrane update rounds after every
// operation, exactly as specified.
#include <algorithm>
#include <type_traits>

#include "snn_internal.h"

namespace snn {

// ---------------------------------------------------------------------------
// helpers

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor S-box with a Weyl-bumped key.  Each product is written as one
// 32x32->64 multiply so that it maps to a single v_mad_u64_u32 (high and low
// halves together) instead of separate mul_hi / mul_lo instructions.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = static_cast<uint64_t>(0xD2511F53u) * c0;
    const uint64_t p1 = static_cast<uint64_t>(0xCD9E8D57u) * c2;
    const uint32_t n0 = static_cast<uint32_t>(p1 >> 32) ^ c1 ^ k0;
    const uint32_t n2 = static_cast<uint32_t>(p0 >> 32) ^ c3 ^ k1;
    c0 = n0;
    c1 = static_cast<uint32_t>(p1);
    c2 = n2;
    c3 = static_cast<uint32_t>(p0);
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return make_uint4(c0, c1, c2, c3);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  return v;
}

// Weight of synapse e.  The kernels that read weights are instantiated per
// weight type, so a BF16 load is never followed by a widening inside a
// run-time branch (which would make each 16-bit load wait for every load in
// flight before the next is issued).
template <bool BF16>
__device__ __forceinline__ float load_weight(const KParams& p, uint64_t e) {
  if constexpr (BF16) {
    const uint16_t b = static_cast<const uint16_t*>(p.weight)[e];
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
  } else {
    return static_cast<const float*>(p.weight)[e];
  }
}

// XCD (XCC) the calling wave runs on: hardware register XCC_ID, bits 3:0.
__device__ __forceinline__ uint32_t xcc_id() {
  return __builtin_amdgcn_s_getreg((31 << 11) | 20) & 0xFu;
}

// Adds the block's sum of two per-thread counters into two global u64s with
// one atomic each per block (atomics on one address serialise, so a block
// sums first).  Every thread of the block calls it; s_red holds 2 * waves.
__device__ void add_stats(uint64_t* dst0, uint64_t v0, uint64_t* dst1, uint64_t v1,
                          uint64_t* s_red) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  v0 = wave_sum64(v0);
  v1 = wave_sum64(v1);
  __syncthreads();
  if (lane == 0) {
    s_red[2 * wave] = v0;
    s_red[2 * wave + 1] = v1;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t a = 0, b = 0;
    for (uint32_t w = 0; w < nw; ++w) {
      a += s_red[2 * w];
      b += s_red[2 * w + 1];
    }
    if (a && dst0) atomicAdd(reinterpret_cast<unsigned long long*>(dst0), a);
    if (b && dst1) atomicAdd(reinterpret_cast<unsigned long long*>(dst1), b);
  }
}

__device__ __forceinline__ void add_stat(uint64_t* dst, uint64_t v, uint64_t* s_red) {
  add_stats(dst, v, nullptr, 0, s_red);
}

// This block's copy of the counters of step row `row`.
__device__ __forceinline__ uint64_t* stat_copy(const KParams& p, uint32_t row) {
  const uint32_t b = blockIdx.y * gridDim.x + blockIdx.x;
  return p.stats + static_cast<uint64_t>(row) * STAT_ROW_WORDS + (b % STAT_LANES) * STAT_LANE_WORDS;
}

// Exclusive prefix sum of one value per thread over the block; *total gets
// the block total.  s_wsum holds one word per wave.  Every thread calls it.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t* s_wsum, uint32_t* total) {
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const uint32_t incl = wave_incl_scan(v);
  __syncthreads();
  if (lane == 63) s_wsum[wave] = incl;
  __syncthreads();
  uint32_t before = 0, tot = 0;
  for (uint32_t w = 0; w < nw; ++w) {
    const uint32_t x = s_wsum[w];
    before += w < wave ? x : 0u;
    tot += x;
  }
  *total = tot;
  return before + incl - v;
}

// Largest k < n with pre[k] <= e, for a non-decreasing pre with pre[0] = 0:
// the segment that holds element e of a concatenation whose segment starts
// are pre.  TOP is a power of two with 2 * TOP >= n (the steps reach 2 * TOP - 1).
template <uint32_t TOP>
__device__ __forceinline__ uint32_t owner_of(const uint32_t* pre, uint32_t n, uint32_t e) {
  uint32_t k = 0;
#pragma unroll
  for (uint32_t step = TOP; step; step >>= 1) {
    const uint32_t m = k + step;
    if (m < n && pre[m] <= e) k = m;
  }
  return k;
}

// Weight in fixed point (multiples of 2^-F, rounded to nearest even; the
// scaling by a power of two is exact) and back.
__device__ __forceinline__ int32_t quantize_w(const KParams& p, float w) {
  return __float2int_rn(w * p.wq_scale);
}
__device__ __forceinline__ float dequantize_w(const KParams& p, int32_t q) {
  return static_cast<float>(static_cast<double>(q) * p.wq_inv);
}

// Tile of neuron x (x < 2^27) by one multiply: floor(x / T).
__device__ __forceinline__ uint32_t tile_of(const KParams& p, uint32_t x) {
  return __umulhi(x, p.tile_magic) >> p.tile_shift;
}

// An event that does not fit its bin goes to the dense overflow ring, which
// holds fixed-point sums (integer atomics: exact in any order, like the
// update's own sums); the tile is flagged so the update reads that slice.
__device__ void ring_fallback(const KParams& p, uint32_t slot, uint32_t tgt, int32_t wq) {
  atomicAdd(p.ovf + slot * p.ring_stride + tgt, wq);
  p.dirty[slot * p.n_tiles + tile_of(p, tgt)] = 1u;
  atomicAdd(reinterpret_cast<unsigned long long*>(&p.st->ring_events), 1ull);
}

// Count index of sub-bin (slot, tile, delay d in 1..max_delay, deliver block
// w): a tile's counts are adjacent (the update reads them in one load).
__device__ __forceinline__ uint64_t subbin(const KParams& p, uint32_t slot, uint32_t tile,
                                           uint32_t d, uint32_t w) {
  const uint32_t md = p.D - 1;
  return ((static_cast<uint64_t>(slot) * p.n_tiles + tile) * md + (d - 1)) * DELIVER_BLOCKS + w;
}

// First event of sub-bin (slot, tile, dw = (d - 1) * DELIVER_BLOCKS + w): the
// sub-bins one deliver block writes, (slot, d, w) over all tiles, are
// adjacent, so its tile-ordered runs land close together.
__device__ __forceinline__ uint64_t bin_data(const KParams& p, uint32_t slot, uint32_t tile,
                                             uint32_t dw) {
  const uint64_t per_slot = static_cast<uint64_t>(p.D - 1) * DELIVER_BLOCKS;
  return ((slot * per_slot + dw) * p.n_tiles + tile) * p.bin_cap;
}

// Sub-bins per (slot, tile) at most.
constexpr uint32_t MAX_SUBBINS = SNN_MAX_DELAY * DELIVER_BLOCKS;
static_assert(MAX_SUBBINS <= UPDATE_THREADS, "one sub-bin count per thread");
constexpr int GATHER_UNROLL = 8;          // loads in flight per thread (deliver, receive)
// The update reads its sub-bins in groups of ARRIVE_LANES lanes, one sub-bin
// per group at a time (lane j takes event j), ARRIVE_UNROLL sub-bins per
// group in flight.
constexpr uint32_t ARRIVE_LANES = 32;
constexpr uint32_t ARRIVE_GROUPS = UPDATE_THREADS / ARRIVE_LANES;
constexpr int ARRIVE_UNROLL = 10;
constexpr int ROUTE_UNROLL = 8;           // destination-list loads in flight per thread
// Two-level routing inside the update kernel (one tile's fired neurons per
// block): the node count up to which its counters fit the LDS the update
// leaves free, and destination-list loads in flight per thread (the window
// of pairs is sized per network, fused_window).
constexpr uint32_t FUSED_MAX_NODES = 512;
constexpr int FUSED_ROUTE_UNROLL = 3;

// ---------------------------------------------------------------------------
// route

// Node of partition v (v < 2^16, G <= 64): v / G as one high multiply; with
// M = ceil(2^32 / G) the product exceeds v / G by less than 2^-16, too little
// to pass the next integer.
__device__ __forceinline__ uint32_t node_of(const KParams& p, uint32_t v) {
  return p.G == 1 ? v : __umulhi(v, p.g_magic);
}

// Mask of node `node`'s destination partitions in s's list from position j
// (the node's first) on: bit b <-> partition G * node + b.
__device__ __forceinline__ uint64_t node_mask(const KParams& p, int64_t j, int64_t j1,
                                              uint32_t node) {
  uint64_t mask = 0;
  for (int64_t jj = j; jj < j1; ++jj) {
    const uint32_t vv = p.vp_part[jj];
    if (node_of(p, vv) != node) break;
    mask |= uint64_t(1) << (vv - p.G * node);
  }
  return mask;
}

// A message in a node's bucket is two words: source | pair index of the
// node's first destination (the receive record the expansion hands on, its
// followers are the next pairs) << 32, then the 64-bit partition mask.
__device__ __forceinline__ void bucket_put(const KParams& p, uint32_t node, uint32_t pos,
                                           uint64_t src_pair, uint64_t mask) {
  const uint64_t off = p.bucket_off[node];
  if (off + pos < p.bucket_off[node + 1]) {
    uint64_t* m = p.bucket + 2 * (off + pos);
    m[0] = src_pair;
    m[1] = mask;
  } else {
    atomicOr(&p.st->error, ERR_BUCKET);
  }
}

// Bucket counters of the step with parity par (t mod 2).  Steps alternate
// between two sets: the update kernel of step t clears the set of step t + 1
// while step t's routing (possibly in the same kernel) counts into its own.
__device__ __forceinline__ uint32_t* bucket_counts(const KParams& p, uint32_t par) {
  return p.bucket_cnt + static_cast<uint64_t>(par) * p.n_nodes * CNT_STRIDE;
}

// LDS arrays of the two-level routing of a batch of at most NT sources of
// one block, over windows of W (source, destination) pairs.  Narrow masks
// (groups of at most 8) travel inside the staged message word; wide ones
// (up to 64) in an array of their own.
struct RouteLds {
  int64_t* j0;     // [NT] first pair index of each source
  uint64_t* msg;   // [W] staged messages: source | list position << 32 (| mask << 48, narrow)
  uint64_t* mask;  // [W] their masks (wide only)
  uint64_t* base;  // [n_nodes] start reserved for the window's messages in each bucket
  uint64_t* end;   // [n_nodes] end of each bucket
  uint32_t* pre;   // [NT + 1] list starts in the concatenation of the batch's lists
  uint32_t* src;   // [NT] source ids of the batch
  uint32_t* nr;    // [W] node | rank among the window's messages to that node << 16
  uint32_t* cnt;   // [n_nodes] messages of the window per node
  uint16_t* own;   // [NT] node of each source
  uint16_t* nb;    // [W] destination partition of each pair
  uint16_t* pk;    // [W] batch index of each pair's source
  uint16_t* off;   // [W] position of each pair in its source's list
  uint16_t* mk;    // [W] batch index of each message's source
  uint32_t W;
};

__host__ __device__ constexpr size_t route_lds_bytes(uint32_t nt, uint32_t w, uint32_t n_nodes,
                                                     bool wide) {
  return 8 * (size_t(nt) + w + (wide ? w : 0) + 2 * size_t(n_nodes)) +
         4 * (2 * size_t(nt) + 1 + w + n_nodes) + 2 * (size_t(nt) + 4 * size_t(w));
}

__device__ RouteLds route_lds(void* lds, uint32_t nt, uint32_t w, uint32_t n_nodes, bool wide) {
  RouteLds L;
  char* c = static_cast<char*>(lds);
  L.j0 = reinterpret_cast<int64_t*>(c);                  c += size_t(nt) * 8;
  L.msg = reinterpret_cast<uint64_t*>(c);                c += size_t(w) * 8;
  L.mask = reinterpret_cast<uint64_t*>(c);               c += wide ? size_t(w) * 8 : 0;
  L.base = reinterpret_cast<uint64_t*>(c);               c += size_t(n_nodes) * 8;
  L.end = reinterpret_cast<uint64_t*>(c);                c += size_t(n_nodes) * 8;
  L.pre = reinterpret_cast<uint32_t*>(c);                c += (size_t(nt) + 1) * 4;
  L.src = reinterpret_cast<uint32_t*>(c);                c += size_t(nt) * 4;
  L.nr = reinterpret_cast<uint32_t*>(c);                 c += size_t(w) * 4;
  L.cnt = reinterpret_cast<uint32_t*>(c);                c += size_t(n_nodes) * 4;
  L.own = reinterpret_cast<uint16_t*>(c);                c += size_t(nt) * 2;
  L.nb = reinterpret_cast<uint16_t*>(c);                 c += size_t(w) * 2;
  L.pk = reinterpret_cast<uint16_t*>(c);                 c += size_t(w) * 2;
  L.off = reinterpret_cast<uint16_t*>(c);                c += size_t(w) * 2;
  L.mk = reinterpret_cast<uint16_t*>(c);
  L.W = w;
  return L;
}

// Group sizes up to which the staged message word carries the mask.
constexpr uint32_t NARROW_G = 8;

// Two-level routing (Sec. IV-B) of the n <= NT sources in L.src: one message
// per (source, destination node) into the node buckets counted by bcnt.
// The sources' destination lists are taken as one flat sequence of pairs: one
// thread per source loads the list bounds, a block scan concatenates the
// lists, and windows of W pairs are loaded into LDS, U loads in flight per
// thread, each pair stored as its partition.  A pair that starts a run of
// equal node in its source's (ascending) list ORs the run into the mask: the
// run has at most G pairs; narrow groups read the next NARROW_G - 1 pairs at
// once from LDS, wide ones walk the run (global memory only for a run that
// continues past the window's end).  Messages are staged in LDS with their
// rank among the window's messages to their node; one atomic per (window,
// node) then reserves the node's bucket space.  A window has at most as many
// messages as pairs, so the stage never overflows.  Every thread of the block
// calls it; it ends with a barrier.
// PRE: the caller may have loaded a source's list bounds and node already:
// then L.j0 holds j0 | len << 32 with bit 63 set and L.own its node (L.j0
// of the other sources is non-negative).
template <uint32_t NT, int U, bool WIDE, bool PRE = false>
__device__ void route_batch(const KParams& p, const RouteLds& L, uint32_t n, uint32_t* bcnt,
                            uint64_t& l1, uint64_t& l2) {
  __shared__ uint32_t l_total, s_prev_node;
  __shared__ uint32_t s_wsum[NT / 64];
  const uint32_t tid = threadIdx.x;
  const uint32_t G = p.G;
  uint32_t len = 0;
  if (tid < n) {
    const int64_t pre = PRE ? L.j0[tid] : 0;
    if (pre < 0) {
      const uint64_t v = static_cast<uint64_t>(pre);
      L.j0[tid] = static_cast<int64_t>(v & 0xFFFFFFFFull);
      len = static_cast<uint32_t>(v >> 32) & 0x7FFFFFFFu;
    } else {
      const uint32_t s = L.src[tid];
      const int64_t j0 = p.vp_ptr[s], j1 = p.vp_ptr[s + 1];
      L.own[tid] = static_cast<uint16_t>(node_of(p, static_cast<uint32_t>(p.part[s])));
      L.j0[tid] = j0;
      len = static_cast<uint32_t>(j1 - j0);
    }
  }
  uint32_t tot;
  const uint32_t ex = block_excl_scan(len, s_wsum, &tot);
  L.pre[tid] = ex;
  if (tid == 0) L.pre[n] = tot;
  __syncthreads();
  for (uint32_t w0 = 0; w0 < tot; w0 += L.W) {
    const uint32_t nwin = min(tot - w0, L.W);
    for (uint32_t i = tid; i < p.n_nodes; i += NT) L.cnt[i] = 0;
    if (tid == 0) {
      l_total = 0;
      // node of the pair before the window, where the window starts inside a list
      const uint32_t k0 = owner_of<NT / 2>(L.pre, n, w0);
      const uint32_t off0 = w0 - L.pre[k0];
      s_prev_node = off0 > 0 ? node_of(p, p.vp_part[L.j0[k0] + off0 - 1]) : 0xFFFFFFFFu;
    }
    // the window's pairs into LDS
    for (uint32_t i0 = 0; i0 < nwin; i0 += U * NT) {
      uint32_t vp[U], kk[U], o[U];
#pragma unroll
      for (int v = 0; v < U; ++v) {
        const uint32_t e = w0 + min(i0 + v * NT + tid, nwin - 1);
        kk[v] = owner_of<NT / 2>(L.pre, n, e);
        o[v] = e - L.pre[kk[v]];
        vp[v] = p.vp_part[L.j0[kk[v]] + o[v]];
      }
#pragma unroll
      for (int v = 0; v < U; ++v) {
        const uint32_t i = i0 + v * NT + tid;
        if (i < nwin) {
          L.nb[i] = static_cast<uint16_t>(vp[v]);
          L.pk[i] = static_cast<uint16_t>(kk[v]);
          L.off[i] = static_cast<uint16_t>(o[v]);
        }
      }
    }
    __syncthreads();
    // one message per run of equal node
    for (uint32_t i = tid; i < nwin; i += NT) {
      const uint32_t k = L.pk[i], off = L.off[i], v0 = L.nb[i];
      const uint32_t node = node_of(p, v0);
      if (off > 0 && (i > 0 ? node_of(p, L.nb[i - 1]) : s_prev_node) == node) continue;
      uint64_t mask = uint64_t(1) << (v0 - G * node);
      bool cut = false;
      if constexpr (!WIDE) {
        bool open = true;
#pragma unroll
        for (uint32_t d = 1; d < NARROW_G; ++d) {
          const bool in = i + d < nwin;
          cut = cut || (open && !in);
          const uint32_t at = min(i + d, nwin - 1);
          const uint32_t v = L.nb[at], kv = L.pk[at];
          open = open && in && kv == k && node_of(p, v) == node;
          if (open) mask |= uint64_t(1) << (v - G * node);
        }
      } else {
        for (uint32_t d = 1; d < G; ++d) {
          if (i + d >= nwin) {
            cut = true;
            break;
          }
          const uint32_t v = L.nb[i + d];
          if (L.pk[i + d] != k || node_of(p, v) != node) break;
          mask |= uint64_t(1) << (v - G * node);
        }
      }
      if (cut) {   // the run reaches the window's end: its rest from global memory
        const uint32_t len_k = L.pre[k + 1] - L.pre[k];
        for (uint32_t x = off + (nwin - i); x < len_k; ++x) {
          const uint32_t v = p.vp_part[L.j0[k] + x];
          if (node_of(p, v) != node) break;
          mask |= uint64_t(1) << (v - G * node);
        }
      }
      const uint32_t slot = atomicAdd(&l_total, 1u);
      const uint32_t rk = atomicAdd(&L.cnt[node], 1u);
      const uint64_t msg = (static_cast<uint64_t>(off) << 32) | L.src[k];
      if constexpr (WIDE) {
        L.msg[slot] = msg;
        L.mask[slot] = mask;
      } else {
        L.msg[slot] = msg | (mask << 48);
      }
      L.nr[slot] = node | (rk << 16);
      L.mk[slot] = static_cast<uint16_t>(k);
      if (node == L.own[k]) ++l1; else ++l2;
    }
    __syncthreads();
    // reservations, with the bucket bounds loaded alongside (same round trip)
    for (uint32_t nn = tid; nn < p.n_nodes; nn += NT) {
      const uint32_t c = L.cnt[nn];
      if (c) {
        const uint64_t o = p.bucket_off[nn], o1 = p.bucket_off[nn + 1];
        L.base[nn] = o + atomicAdd(bcnt + nn * CNT_STRIDE, c);
        L.end[nn] = o1;
      }
    }
    __syncthreads();
    const uint32_t n_msg = l_total;
    for (uint32_t k = tid; k < n_msg; k += NT) {
      const uint32_t nr = L.nr[k];
      const uint32_t node = nr & 0xFFFFu;
      const uint64_t pos = L.base[node] + (nr >> 16);
      if (pos < L.end[node]) {
        const uint64_t msg = L.msg[k];
        const uint64_t pair = static_cast<uint64_t>(L.j0[L.mk[k]]) + ((msg >> 32) & 0xFFFFu);
        p.bucket[2 * pos] = (msg & 0xFFFFFFFFull) | (pair << 32);
        p.bucket[2 * pos + 1] = WIDE ? L.mask[k] : msg >> 48;
      } else {
        atomicOr(&p.st->error, ERR_BUCKET);
      }
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// update: arriving input, neuron update, threshold, ascending compaction

// Look-back word: [63:34] step tag, [33:32] status, [31:0] count.
constexpr uint32_t LB_AGG = 1u, LB_INCL = 2u;

__device__ __forceinline__ uint64_t lb_pack(uint32_t tag, uint32_t status, uint32_t v) {
  return (static_cast<uint64_t>(tag) << 34) | (static_cast<uint64_t>(status) << 32) | v;
}

// Decoupled look-back, run by wave 0 of block b in two parts so that a block
// can do other work between them: lookback_publish makes the block's count
// visible (block 0 publishes its inclusive prefix at once), lookback_resolve
// walks back over the predecessors 64 at a time until an inclusive prefix
// closes the window, publishes the block's inclusive prefix and returns the
// exclusive one.
// The 64-bit word carries tag, status and count together and nothing else
// is read through it, so relaxed device-scope atomics suffice: acquire or
// release would add an L2 invalidate or write-back to every poll.
__device__ void lookback_publish(uint64_t* lb, uint32_t b, uint32_t agg, uint32_t tag) {
  if ((threadIdx.x & 63) == 0)
    __hip_atomic_store(lb + b, lb_pack(tag, b == 0 ? LB_INCL : LB_AGG, agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
}

__device__ uint32_t lookback_resolve(uint64_t* lb, uint32_t b, uint32_t agg, uint32_t tag) {
  const int lane = threadIdx.x & 63;
  if (b == 0) return 0;
  uint32_t excl = 0;
  int64_t j = static_cast<int64_t>(b) - 1;
  while (true) {
    const int64_t idx = j - lane;
    uint64_t w = idx >= 0 ? __hip_atomic_load(lb + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                          : lb_pack(tag, LB_INCL, 0);
    const uint32_t status = static_cast<uint32_t>(w >> 32) & 3u;
    const bool ready = static_cast<uint32_t>(w >> 34) == tag && status != 0;
    const uint64_t incl = __ballot(ready && status == LB_INCL);
    const uint64_t notready = __ballot(!ready);
    if (incl) {
      const int f = __ffsll(static_cast<unsigned long long>(incl)) - 1;
      const uint64_t upto = f == 63 ? ~0ull : ((2ull << f) - 1);
      if (notready & upto) {
        __builtin_amdgcn_s_sleep(1);
        continue;
      }
      excl += wave_sum(lane <= f ? static_cast<uint32_t>(w) : 0u);
      break;
    }
    if (notready) {
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    excl += wave_sum(static_cast<uint32_t>(w));
    j -= 64;
  }
  if (lane == 0)
    __hip_atomic_store(lb + b, lb_pack(tag, LB_INCL, excl + agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// One block per tile.  Thread tid owns UPDATE_NPT neurons as UPDATE_NPT / 4
// quads: quad q covers tile neurons q*4*UPDATE_THREADS + 4*tid .. +3, so
// every load and store instruction of a wave touches one contiguous 1 KiB
// span.  Ids are ordered quad-major across the block, which the compaction
// follows.
// With ROUTE, the block also routes its tile's fired neurons two-level
// (route_batch) between publishing its spike count and resolving its prefix,
// so the routing's latency overlaps the look-back and no separate routing
// launch is needed; the LDS of the input sums and the Poisson lookup, free by
// then, holds the routing's arrays.
static_assert(UPDATE_NPT % 4 == 0 && UPDATE_NPT <= 32, "fire bits of a thread fit 32 bits");
// The input sums and the Poisson lookup, plus room that lets the routing's
// window hold a tile's usual fired neurons at once (three blocks per CU still
// fit the CU's LDS).
constexpr size_t UPDATE_BIG_LDS = TILE_MAX * sizeof(int32_t) + POIS_LUT_SIZE + 4096;
// Pairs per routing window inside the update: as many as fit UPDATE_BIG_LDS
// beside the per-source and per-node arrays of n_nodes nodes (a multiple of
// 64).  On the share (250 nodes) 1,536 pairs, about eight sources' lists, so
// that a tile's fired neurons (about four) are routed in one window.
__host__ __device__ constexpr uint32_t fused_window(uint32_t n_nodes) {
  const size_t fixed = route_lds_bytes(UPDATE_THREADS, 0, n_nodes, false);
  const size_t per_pair = route_lds_bytes(UPDATE_THREADS, 1, n_nodes, false) - fixed;
  return static_cast<uint32_t>((UPDATE_BIG_LDS - fixed) / per_pair) / 64 * 64;
}
static_assert(fused_window(FUSED_MAX_NODES) >= 1024, "the fused routing's arrays fit the update's LDS");
// PERSIST: a grid smaller than the launch's tiles, whose blocks take further
// tiles by ticket (a separate instantiation: the loop carried across tiles
// costs registers, 106 VGPRs against 73, so two blocks per CU instead of
// three).
template <bool ROUTE, bool PERSIST>
__global__ __launch_bounds__(UPDATE_THREADS) void k_update(KParams p) {
  constexpr int NQ = UPDATE_NPT / 4;
  constexpr int NW = UPDATE_THREADS / 64;
  // input sums (T int32, fixed point in units of 2^-F) and the Poisson
  // inversion lookup (bytes); the routing's arrays afterwards
  __shared__ uint4 s_big[UPDATE_BIG_LDS / 16];
  int32_t* s_acc = reinterpret_cast<int32_t*>(s_big);
  uint4* s_lut4 = s_big + TILE_MAX / 4;
  __shared__ uint32_t s_cnt[NQ][NW];    // spikes per (quad, wave)
  __shared__ uint32_t s_qoff[NQ][NW];   // their offsets in the block's order
  __shared__ uint32_t s_bcnt[MAX_SUBBINS];
  __shared__ uint32_t s_excl, s_btot;
  __shared__ uint32_t s_dirty;
  __shared__ uint32_t s_thr[16];
  __shared__ uint64_t s_red[2 * NW];

  // Read once (uniform, so kept in scalar registers): the last block advances
  // the step state when the step is complete.
  const DevState* st = p.st;
  auto rd32 = [](const uint32_t* a) {
    return __builtin_amdgcn_readfirstlane(
        __hip_atomic_load(a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  };
  const uint32_t t32 = rd32(reinterpret_cast<const uint32_t*>(&st->t));   // low word
  const uint32_t slot = rd32(&st->slot);
  const uint32_t row = rd32(&st->row);
  const uint32_t srow = rd32(&st->srow);
  const uint32_t phase = rd32(&st->phase);
  const uint32_t tag = rd32(&st->tag) + 1u;
  const uint64_t log_head =
      (static_cast<uint64_t>(rd32(reinterpret_cast<const uint32_t*>(&st->log_head) + 1)) << 32) |
      rd32(reinterpret_cast<const uint32_t*>(&st->log_head));
  // fired ids of the step's earlier launches (one launch per partition)
  const uint32_t base = rd32(&st->part_base);
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  __shared__ uint32_t s_tile;
  // The launch covers tiles [tile0, tile_end) and neurons [lo, hi).  Block b
  // takes tile tile0 + b; a grid smaller than that (persistent) takes the
  // rest in ticket order, so the look-back only ever waits for tiles already
  // taken by running blocks.
  uint32_t tile = p.tile0 + blockIdx.x;
  while (true) {
  const uint32_t T = p.tile;
  const uint32_t blk0 = tile * T;
  // the neurons of this tile the launch updates
  const uint32_t lo_t = max(p.lo, blk0), hi_t = min(p.hi, blk0 + T);

  // Per-step counters of the routing: the bucket counters of step t + 1 (this
  // step's routing counts into the other set) and the receive-list counters.
  if (tile == 0) {
    if (tid == 0) p.tickets[(t32 + 1u) & 1u] = 0u;
    uint32_t* next_bcnt = bucket_counts(p, (t32 + 1u) & 1u);
    for (uint32_t i = tid; i < p.n_nodes; i += UPDATE_THREADS) next_bcnt[i * CNT_STRIDE] = 0;
    for (uint32_t i = tid; i < p.P; i += UPDATE_THREADS) {
      p.recv_cnt[i * CNT_STRIDE] = 0;
      p.flat_cnt[i * CNT_STRIDE] = 0;
    }
    // the counter row of step t + 1 (this step's was cleared by the step before)
    const uint32_t next_srow = srow + 1 == p.log_steps + 1 ? 0u : srow + 1;
    if (tid < STAT_ROW_WORDS) p.stats[static_cast<uint64_t>(next_srow) * STAT_ROW_WORDS + tid] = 0;
  }
  // the tile's sub-bin counts (one coalesced load), issued first so that
  // their latency overlaps the set-up below
  const uint32_t md = p.D - 1;
  const uint32_t n_sub = md * DELIVER_BLOCKS;
  const uint32_t bc_raw = tid < n_sub ? p.bin_cnt[subbin(p, slot, tile, 1, 0) + tid] : 0u;
  for (uint32_t i = tid; i < T; i += UPDATE_THREADS) s_acc[i] = 0;
  if (tid == 0) s_dirty = p.dirty[slot * p.n_tiles + tile];
  for (uint32_t i = tid; i < POIS_LUT_SIZE / 16; i += UPDATE_THREADS)
    s_lut4[i] = reinterpret_cast<const uint4*>(p.pois_lut)[i];
  if (tid < 15) s_thr[tid] = p.thr[tid];
  const uint8_t* s_lut = reinterpret_cast<const uint8_t*>(s_lut4);

  // State of quad q of the thread's neurons (4 consecutive neurons; T is a
  // multiple of 4, so a quad lies inside the tile or past its end).  The
  // branch on a whole tile in range is uniform, so loads carry no divergent
  // merge; past the launch's range a lane reads an in-range neuron (never
  // stored back, never fires); quads past the tile's end load nothing.
  const bool tile_full = lo_t == blk0 && hi_t == blk0 + T;
  auto load_quad = [&](int q, float4& u4, uint32_t& r4) {
    const uint32_t l0 = q * (4 * UPDATE_THREADS) + 4 * tid;
    const uint32_t i0 = blk0 + l0;
    if (l0 >= T) {
      u4 = make_float4(0.f, 0.f, 0.f, 0.f);
      r4 = 0;
    } else if (tile_full) {
      u4 = *reinterpret_cast<const float4*>(p.u + i0);
      r4 = *reinterpret_cast<const uint32_t*>(p.ref + i0);
    } else {
      float v[4];
      uint32_t r = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t ik = min(max(i0 + k, lo_t), hi_t - 1);
        v[k] = p.u[ik];
        r |= static_cast<uint32_t>(p.ref[ik]) << (8 * k);
      }
      u4 = make_float4(v[0], v[1], v[2], v[3]);
      r4 = r;
    }
  };
  // quad 0 is loaded now so that its loads overlap the gather
  float4 u_next;
  uint32_t r_next;
  load_quad(0, u_next, r_next);
  __syncthreads();

  // Arriving input of step t: the sub-bins (slot, tile, d, w) written d steps
  // ago by deliver block w.  Their counts are read in one coalesced load;
  // then each group of ARRIVE_LANES lanes takes whole sub-bins, so an event's
  // address is its sub-bin's start plus the lane (no search over the counts).
  // A lane without an event re-reads event 0 of the tile's first sub-bin (a
  // valid address) and skips the add, so the loads carry no branch and issue
  // together.  Events past ARRIVE_LANES in a sub-bin (rare) take a second loop.
  if (tid < n_sub) s_bcnt[tid] = min(bc_raw, static_cast<uint32_t>(p.bin_cap));
  __syncthreads();
  // sub-bin dw of this tile starts at ev0 + dw * sub_stride
  const Event* ev0 = p.bins + bin_data(p, slot, tile, 0);
  const uint64_t sub_stride = static_cast<uint64_t>(p.n_tiles) * p.bin_cap;
  const uint32_t grp = tid / ARRIVE_LANES, gl = tid % ARRIVE_LANES;
  bool over = false;
  for (uint32_t k0 = grp; k0 < n_sub; k0 += ARRIVE_GROUPS * ARRIVE_UNROLL) {
    bool has[ARRIVE_UNROLL];
    Event x[ARRIVE_UNROLL];
#pragma unroll
    for (int v = 0; v < ARRIVE_UNROLL; ++v) {
      const uint32_t k = k0 + v * ARRIVE_GROUPS;
      const uint32_t c = k < n_sub ? s_bcnt[k] : 0u;
      has[v] = gl < c;
      over |= c > ARRIVE_LANES;
      x[v] = ev0[has[v] ? k * sub_stride + gl : 0];
    }
#pragma unroll
    for (int v = 0; v < ARRIVE_UNROLL; ++v)
      if (has[v]) atomicAdd(&s_acc[x[v].tgt], x[v].wq);
  }
  if (__syncthreads_or(over)) {
    // the rest of sub-bins with more than ARRIVE_LANES events (bursts), with
    // ARRIVE_UNROLL loads in flight per lane as above
    for (uint32_t k = grp; k < n_sub; k += ARRIVE_GROUPS) {
      const uint32_t c = s_bcnt[k];
      const Event* sb = ev0 + k * sub_stride;
      for (uint32_t j0 = ARRIVE_LANES; j0 < c; j0 += ARRIVE_LANES * ARRIVE_UNROLL) {
        bool has[ARRIVE_UNROLL];
        Event x[ARRIVE_UNROLL];
#pragma unroll
        for (int v = 0; v < ARRIVE_UNROLL; ++v) {
          const uint32_t j = j0 + v * ARRIVE_LANES + gl;
          has[v] = j < c;
          x[v] = sb[has[v] ? j : 0u];
        }
#pragma unroll
        for (int v = 0; v < ARRIVE_UNROLL; ++v)
          if (has[v]) atomicAdd(&s_acc[x[v].tgt], x[v].wq);
      }
    }
    __syncthreads();
  }
  // events that did not fit their bins are in this tile's slice of the
  // overflow ring slot; a flagged tile adds (and clears) it with the neuron
  // state, before the sum is rounded
  int32_t* ovf_slot = p.ovf + static_cast<uint64_t>(slot) * p.ring_stride;
  const bool dirty = s_dirty != 0;
  // (cleared by the launch that holds the tile's last neuron)
  if (dirty && tid == 0 && min(blk0 + T, p.N) <= p.hi) p.dirty[slot * p.n_tiles + tile] = 0u;

  uint32_t thr_raster = 0;
  if (p.forced) thr_raster = phase < p.raster_on ? p.raster_on_thr : p.raster_off_thr;

  uint32_t fire_bits = 0;   // bit 4q + k: neuron k of quad q fired
  // With ROUTE, the list bounds and node of the thread's first fired neuron,
  // loaded as soon as it fires, so that they arrive while the block finishes
  // its other quads and the compaction (the routing then skips that round
  // trip for it).  Pair indices are below 2^32 (checked at create).
  uint32_t pf_id = 0xFFFFFFFFu, pf_part = 0;
  int64_t pf_j0 = 0, pf_j1 = 0;
  // One quad per iteration, the next quad's loads issued before this quad's
  // arithmetic (not unrolled: keeps the kernel within 128 VGPRs, two blocks
  // per CU).
#pragma unroll 1
  for (int q = 0; q < NQ; ++q) {
    const float4 u4 = u_next;
    const uint32_t r4 = r_next;
    if (q + 1 < NQ) load_quad(q + 1, u_next, r_next);
    const uint32_t l0 = q * (4 * UPDATE_THREADS) + 4 * tid;
    const uint32_t i0 = blk0 + l0;
    // Philox counter word 0 is i0 / 4: one call serves the quad's 4 neurons.
    const uint4 rnd = philox4x32_10(i0 >> 2, t32, STREAM_POISSON, 0u, p.seed_lo, p.seed_hi);
    uint4 rnd2 = make_uint4(0, 0, 0, 0);
    if (p.forced) rnd2 = philox4x32_10(i0 >> 2, t32, STREAM_RASTER, 0u, p.seed_lo, p.seed_hi);
    const uint32_t r1[4] = {rnd.x, rnd.y, rnd.z, rnd.w};
    const uint32_t r2[4] = {rnd2.x, rnd2.y, rnd2.z, rnd2.w};
    // arriving input: the exact fixed-point sum (bins, plus the overflow
    // ring slice of a flagged tile) rounded once to binary32 (rounding the
    // integer and then scaling by the power of two 2^-F gives the same
    // value: the scaling is exact)
    const int4 acc4 = *reinterpret_cast<const int4*>(&s_acc[l0]);
    int32_t acc[4] = {acc4.x, acc4.y, acc4.z, acc4.w};
    if (dirty) {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i0 + k >= lo_t && i0 + k < hi_t) {
          acc[k] += ovf_slot[i0 + k];
          ovf_slot[i0 + k] = 0;
        }
    }
    const float wq_inv = static_cast<float>(p.wq_inv);
    float syn[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) syn[k] = __fmul_rn(static_cast<float>(acc[k]), wq_inv);
    float uu[4] = {u4.x, u4.y, u4.z, u4.w};
    uint32_t rf[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) rf[k] = (r4 >> (8 * k)) & 0xFFu;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      // Poisson count k = #{j : thr[j] <= r} through the lookup; ranges
      // holding several thresholds (far tail) count all of them.
      const uint32_t r = r1[k];
      const uint32_t e = s_lut[r >> POIS_LUT_SHIFT];
      const uint32_t j = min(e - 16u, 14u);
      uint32_t kk = e < 16u ? e : j + (r >= s_thr[j] ? 1u : 0u);
      if (e == POIS_LUT_SLOW) {
        kk = 0;
#pragma unroll
        for (int jj = 0; jj < 15; ++jj) kk += p.thr[jj] <= r ? 1u : 0u;
      }
      const float ext = __fmul_rn(static_cast<float>(kk), p.w_ext);
      // integrate unless refractory (then the count drops and u stays):
      // u = fl(fl(u * alpha) + fl(syn + ext)), selected without branches
      const bool integrating = rf[k] == 0;
      const float u_int = __fadd_rn(__fmul_rn(uu[k], p.alpha), __fadd_rn(syn[k], ext));
      const float un = integrating ? u_int : uu[k];
      const uint32_t rn = integrating ? 0u : rf[k] - 1u;
      bool s = p.forced ? (r2[k] < thr_raster) : (integrating && un >= p.theta);
      s = s && (i0 + k >= lo_t && i0 + k < hi_t);
      uu[k] = s ? p.u_reset : un;
      rf[k] = s ? p.n_ref : rn;
      fire_bits |= static_cast<uint32_t>(s) << (4 * q + k);
    }
    uint32_t cnt_q = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) cnt_q += __popcll(__ballot((fire_bits >> (4 * q + k)) & 1u));
    if (lane == 0) s_cnt[q][wave] = cnt_q;
    if constexpr (ROUTE) {
      const uint32_t qb = (fire_bits >> (4 * q)) & 0xFu;
      if (qb && pf_id == 0xFFFFFFFFu) {
        pf_id = i0 + static_cast<uint32_t>(__ffs(qb) - 1);
        pf_j0 = p.vp_ptr[pf_id];
        pf_j1 = p.vp_ptr[pf_id + 1];
        pf_part = static_cast<uint32_t>(p.part[pf_id]);
      }
    }
    if (tile_full) {
      if (l0 < T) {
        *reinterpret_cast<float4*>(p.u + i0) = make_float4(uu[0], uu[1], uu[2], uu[3]);
        *reinterpret_cast<uint32_t*>(p.ref + i0) =
            rf[0] | (rf[1] << 8) | (rf[2] << 16) | (rf[3] << 24);
      }
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i0 + k >= lo_t && i0 + k < hi_t) {
          p.u[i0 + k] = uu[k];
          p.ref[i0 + k] = static_cast<uint8_t>(rf[k]);
        }
    }
  }

  // Compaction.  Within quad q, ids ascend with (wave, lane, k); across
  // quads, quad q of every wave precedes quad q + 1.  The rank of a fired id
  // in the block is: the offset of its (quad, wave) in that order (one wave
  // scans the NQ x NW counts) + fired ids of lower lanes in the same (quad,
  // wave) (4 ballots) + earlier k.  The block's total goes through the
  // look-back.
  static_assert(NQ * NW <= 64, "one lane per (quad, wave)");
  __syncthreads();
  if (wave == 0) {
    const uint32_t c = lane < NQ * NW ? s_cnt[lane / NW][lane % NW] : 0u;
    const uint32_t incl = wave_incl_scan(c);
    if (lane < NQ * NW) s_qoff[lane / NW][lane % NW] = incl - c;
    const uint32_t block_tot = __shfl(incl, 63, 64);
    lookback_publish(p.lookback, tile - p.tile0, block_tot, tag);
    if (lane == 0) s_btot = block_tot;
  }
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  // f(rank in the block, id) for every fired neuron of this thread
  auto for_each_fired = [&](auto&& f) {
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      const uint32_t qb = (fire_bits >> (4 * q)) & 0xFu;
      if (__ballot(qb != 0) == 0) continue;
      uint32_t pos = s_qoff[q][wave];
#pragma unroll
      for (int k = 0; k < 4; ++k) pos += __popcll(__ballot((qb >> k) & 1u) & lt);
      const uint32_t i0 = blk0 + q * (4 * UPDATE_THREADS) + 4 * tid;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((qb >> k) & 1u) f(pos++, i0 + k);
    }
  };
  const uint32_t btot = s_btot;

  if constexpr (ROUTE) {
    // the tile's fired neurons, UPDATE_THREADS at a time, routed into the
    // bucket set of this step
    const RouteLds L = route_lds(s_big, UPDATE_THREADS, fused_window(p.n_nodes), p.n_nodes, false);
    uint32_t* bcnt = bucket_counts(p, t32 & 1u);
    uint64_t l1 = 0, l2 = 0;
    for (uint32_t b0 = 0; b0 < btot; b0 += UPDATE_THREADS) {
      for_each_fired([&](uint32_t r, uint32_t id) {
        if (r - b0 < UPDATE_THREADS) {
          L.src[r - b0] = id;
          if (id == pf_id) {
            L.j0[r - b0] = static_cast<int64_t>(static_cast<uint64_t>(pf_j0) |
                                                (static_cast<uint64_t>(pf_j1 - pf_j0) << 32) |
                                                (uint64_t(1) << 63));
            L.own[r - b0] = static_cast<uint16_t>(node_of(p, pf_part));
          } else {
            L.j0[r - b0] = 0;
          }
        }
      });
      __syncthreads();
      route_batch<UPDATE_THREADS, FUSED_ROUTE_UNROLL, false, true>(
          p, L, min(btot - b0, static_cast<uint32_t>(UPDATE_THREADS)), bcnt, l1, l2);
    }
    uint64_t* sc = stat_copy(p, srow);
    add_stats(sc + SNN_STAT_MSG_L1, l1, sc + SNN_STAT_MSG_L2, l2, s_red);
  }

  if (wave == 0) {
    const uint32_t excl = lookback_resolve(p.lookback, tile - p.tile0, btot, tag);
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  const uint32_t excl = s_excl;
  for_each_fired([&](uint32_t r, uint32_t id) {
    const uint32_t pos = base + excl + r;
    p.fired[pos] = id;
    // a step with more spikes than the log holds is flagged by the last
    // block (ERR_LOG); its ids past the capacity are not logged
    if (pos < p.log_cap) {
      uint64_t at = log_head + pos;
      if (at >= p.log_cap) at -= p.log_cap;
      p.log[at] = id;
    }
  });

  // The launch's last tile holds the launch total once its look-back is done;
  // every other block has read the state by then (they published first).
  // It hands the next launch its look-back tag, and the step's last launch
  // advances the step state.
  if (tile == p.tile_end - 1 && tid == 0) {
    DevState* w = p.st;
    const uint32_t n = base + s_excl + s_btot;
    w->tag = tag == 0x3FFFFFFFu ? 0u : tag;          // next tag - 1 = this tag
    if (!p.step_ends) {
      w->part_base = n;
    } else {
      const uint64_t log_base = w->log_total;
      w->part_base = 0;
      w->n_fired = n;
      p.stats[static_cast<uint64_t>(srow) * STAT_ROW_WORDS + SNN_STAT_SPIKES] = n;
      p.log_off[row] = log_base;
      if (p.log_cap && n > p.log_cap) atomicOr(&w->error, ERR_LOG);
      w->log_total = log_base + n;
      if (p.log_cap) w->log_head = (w->log_head + n) % p.log_cap;
      w->cur_slot = slot;
      w->cur_row = row;
      w->cur_par = t32 & 1u;
      w->cur_srow = srow;
      w->srow = srow + 1 == p.log_steps + 1 ? 0u : srow + 1;
      w->slot = slot + 1 == p.D ? 0u : slot + 1;
      w->row = row + 1 == p.log_steps ? 0u : row + 1;
      w->phase = phase + 1 == p.raster_period ? 0u : phase + 1;
      w->t = w->t + 1;
    }
  }
  if constexpr (!PERSIST) break;                    // one tile per block
  __syncthreads();
  if (tid == 0) s_tile = p.tile0 + gridDim.x + atomicAdd(p.tickets + (t32 & 1u), 1u);
  __syncthreads();
  tile = s_tile;
  if (tile >= p.tile_end) break;
  __syncthreads();
  }   // tiles
}

static_assert(route_lds_bytes(ROUTE_THREADS, ROUTE_STAGE, ROUTE_MAX_NODES_LDS, true) <= 150u * 1024u,
              "the routing kernel's arrays fit a CU's LDS");
static_assert(ROUTE_STAGE <= 65536 && ROUTE_MAX_NODES_LDS <= 8192,
              "ranks and nodes fit their 16-bit fields");

// Two-level routing as a kernel of its own: block b routes a contiguous chunk
// of the step's fired sources, ROUTE_THREADS at a time (route_batch).
// Dynamic LDS: route_lds_bytes(ROUTE_THREADS, ROUTE_STAGE, n_nodes, WIDE).
template <bool WIDE>
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_two_level(KParams p) {
  extern __shared__ uint64_t lds_u64[];
  __shared__ uint64_t s_red[2 * (ROUTE_THREADS / 64)];
  const RouteLds L = route_lds(lds_u64, ROUTE_THREADS, ROUTE_STAGE, p.n_nodes, WIDE);
  const uint32_t nF = p.st->n_fired;
  const uint32_t row = p.st->cur_srow;   // counter row
  uint32_t* bcnt = bucket_counts(p, p.st->cur_par);
  const uint32_t tid = threadIdx.x;
  const uint32_t chunk = (nF + gridDim.x - 1) / gridDim.x;
  const uint32_t lo = min(blockIdx.x * chunk, nF), hi = min(lo + chunk, nF);
  uint64_t l1 = 0, l2 = 0;
  for (uint32_t r0 = lo; r0 < hi; r0 += ROUTE_THREADS) {
    const uint32_t n = min(hi - r0, static_cast<uint32_t>(ROUTE_THREADS));
    if (tid < n) L.src[tid] = p.fired[r0 + tid];
    __syncthreads();
    route_batch<ROUTE_THREADS, ROUTE_UNROLL, WIDE>(p, L, n, bcnt, l1, l2);
  }
  uint64_t* st = stat_copy(p, row);
  add_stats(st + SNN_STAT_MSG_L1, l1, st + SNN_STAT_MSG_L2, l2, s_red);
}

// Two-level routing without LDS staging, for node counts whose counters do
// not fit LDS: one wave per source, one atomic per message.
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_two_level_direct(KParams p) {
  const uint32_t nF = p.st->n_fired;
  uint32_t* bcnt = bucket_counts(p, p.st->cur_par);
  const uint32_t row = p.st->cur_srow;   // counter row
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t n_waves = gridDim.x * (ROUTE_THREADS / 64);
  uint64_t l1 = 0, l2 = 0;
  for (uint32_t i = blockIdx.x * (ROUTE_THREADS / 64) + (threadIdx.x >> 6); i < nF; i += n_waves) {
    const uint32_t s = p.fired[i];
    const uint32_t own_node = node_of(p, static_cast<uint32_t>(p.part[s]));
    const int64_t j0 = p.vp_ptr[s], j1 = p.vp_ptr[s + 1];
    for (int64_t jb = j0; jb < j1; jb += 64) {
      const int64_t j = jb + lane;
      if (j >= j1) continue;
      const uint32_t node = node_of(p, p.vp_part[j]);
      if (j != j0 && node_of(p, p.vp_part[j - 1]) == node) continue;
      bucket_put(p, node, atomicAdd(bcnt + node * CNT_STRIDE, 1u),
                 static_cast<uint64_t>(s) | (static_cast<uint64_t>(j) << 32),
                 node_mask(p, j, j1, node));
      if (node == own_node) ++l1; else ++l2;
    }
  }
  __shared__ uint64_t s_red[2 * (ROUTE_THREADS / 64)];
  uint64_t* st = stat_copy(p, row);
  add_stats(st + SNN_STAT_MSG_L1, l1, st + SNN_STAT_MSG_L2, l2, s_red);
}

// Flat (direct peer-to-peer) routing: one wave per fired source, one receive
// entry (source, pair index) per destination partition.
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_flat(KParams p) {
  const uint32_t nF = p.st->n_fired;
  const uint32_t row = p.st->cur_srow;   // counter row
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t n_waves = gridDim.x * (ROUTE_THREADS / 64);
  uint64_t flat = 0;
  for (uint32_t i = blockIdx.x * (ROUTE_THREADS / 64) + (threadIdx.x >> 6); i < nF; i += n_waves) {
    const uint32_t s = p.fired[i];
    const int64_t j0 = p.vp_ptr[s], j1 = p.vp_ptr[s + 1];
    for (int64_t j = j0 + lane; j < j1; j += 64) {
      const uint32_t v = p.vp_part[j];
      const uint32_t pos = atomicAdd(p.flat_cnt + v * CNT_STRIDE, 1u);
      const uint64_t off = p.recv_off[v];
      if (off + pos < p.recv_off[v + 1])
        p.flat[off + pos] = static_cast<uint64_t>(s) | (static_cast<uint64_t>(j) << ENTRY_SRC_BITS);
      else
        atomicOr(&p.st->error, ERR_FLAT);
      ++flat;
    }
  }
  __shared__ uint64_t s_red[2 * (ROUTE_THREADS / 64)];
  add_stat(stat_copy(p, row) + SNN_STAT_FLAT_MSGS, flat, s_red);
}

// ---------------------------------------------------------------------------
// receive side: stage remote synapses per delay

// A receive-side block's per-delay staging queues and the LDS it stages with.
struct StageCtx {
  Event* queue;        // queue of delay 1 of this block; delay d at + (d - 1) * qstride
  uint64_t qstride;
  uint32_t slot0;      // ring slot of the step in flight
  uint32_t* l_pos;     // [SNN_MAX_DELAY] events queued per delay
  uint64_t* s_seg;     // [RECV_BATCH] second synapse of each entry's segment
  uint32_t* s_epre;    // [RECV_BATCH] remaining synapses: starts in the concatenation
  uint32_t* s_wsum;    // [RECV_THREADS / 64]
};

// One synapse (tgt_delay, weight) into the queue of its delay (position from
// an LDS counter; the queue belongs to the block), or into the dense ring
// when the queue is full.
__device__ __forceinline__ void stage_emit(const KParams& p, const StageCtx& c, uint32_t td,
                                           float w) {
  const uint32_t d1 = (td >> 27) - 1;
  if (d1 >= p.D - 1) {                       // delay outside [1, max_delay]
    atomicOr(&p.st->error, ERR_ROUTE);
    return;
  }
  const Event ev{td & 0x07FFFFFFu, quantize_w(p, w)};
  const uint32_t pos = atomicAdd(&c.l_pos[d1], 1u);
  if (pos < p.stage_cap) {
    c.queue[d1 * c.qstride + pos] = ev;
  } else {
    uint32_t slot = c.slot0 + d1 + 1;
    if (slot >= p.D) slot -= p.D;
    ring_fallback(p, slot, ev.tgt, ev.wq);
  }
}

// Stages the synapses of nb <= RECV_BATCH receive entries, RECV_PER_THREAD
// per thread in ent (entry tid * R + v; lanes past nb hold a valid entry and
// contribute nothing).  An entry (s, j) names the receive record of pair j:
// the row segment of s going to the entry's partition, with its first synapse
// inline.  The two dependent loads (entry, record) of all entries are in
// flight together; the first synapse of every segment comes from the record,
// and the rest of the longer segments are concatenated by a block scan and
// loaded as one flat sequence, GATHER_UNROLL loads in flight per thread.
// Every thread calls it; it ends with a barrier.
template <bool BF16>
__device__ void stage_batch(const KParams& p, const StageCtx& c, const uint64_t* ent, uint32_t nb,
                            uint64_t& events) {
  constexpr uint32_t R = RECV_PER_THREAD;
  const uint32_t tid = threadIdx.x;
  uint64_t rec0[R], rec1[R];
#pragma unroll
  for (int v = 0; v < R; ++v) {
    const uint64_t j = ent[v] >> ENTRY_SRC_BITS;
    const uint64_t jc = j < p.n_pairs ? j : 0;   // entries exist, so pair 0 does
    rec0[v] = p.vp_rec[2 * jc];
    rec1[v] = p.vp_rec[2 * jc + 1];
  }
  uint32_t len[R];
  uint32_t tsum = 0;
#pragma unroll
  for (int v = 0; v < R; ++v) {
    const bool in = tid * R + v < nb;
    const uint64_t start = rec0[v] & ((uint64_t(1) << 40) - 1);
    const uint32_t seg_len = static_cast<uint32_t>(rec0[v] >> 40);
    const bool ok = (ent[v] & ENTRY_SRC_MASK) < p.N && (ent[v] >> ENTRY_SRC_BITS) < p.n_pairs &&
                    seg_len >= 1 && start + seg_len <= p.nnz;
    if (in && !ok) atomicOr(&p.st->error, ERR_ROUTE);
    if (in && ok) {
      const uint32_t wbits = static_cast<uint32_t>(rec1[v] >> 32);
      stage_emit(p, c, static_cast<uint32_t>(rec1[v]),
                 BF16 ? __uint_as_float(wbits << 16) : __uint_as_float(wbits));
      events += seg_len;
    }
    c.s_seg[tid * R + v] = start + 1;
    len[v] = in && ok ? seg_len - 1 : 0u;
    tsum += len[v];
  }
  uint32_t T;
  uint32_t run = block_excl_scan(tsum, c.s_wsum, &T);
#pragma unroll
  for (int v = 0; v < R; ++v) {
    c.s_epre[tid * R + v] = run;
    run += len[v];
  }
  __syncthreads();
  // the remaining synapses of longer segments
  for (uint32_t e0 = 0; e0 < T; e0 += GATHER_UNROLL * RECV_THREADS) {
    uint32_t td[GATHER_UNROLL];
    float wt[GATHER_UNROLL];
#pragma unroll
    for (int v = 0; v < GATHER_UNROLL; ++v) {
      const uint32_t e = min(e0 + v * RECV_THREADS + tid, T - 1);
      const uint32_t k = owner_of<RECV_BATCH / 2>(c.s_epre, nb, e);
      const uint64_t x = c.s_seg[k] + (e - c.s_epre[k]);
      td[v] = p.tgt_delay[x];
      wt[v] = load_weight<BF16>(p, x);
    }
#pragma unroll
    for (int v = 0; v < GATHER_UNROLL; ++v)
      if (e0 + v * RECV_THREADS + tid < T) stage_emit(p, c, td[v], wt[v]);
  }
  __syncthreads();
}

// Receive lists -> staging queues.  Block b of STAGE_BLOCKS owns a contiguous
// range of partitions and their receive lists (expanded or flat), taken in
// batches of RECV_BATCH entries (stage_batch).
template <bool BF16>
__global__ __launch_bounds__(RECV_THREADS) void k_recv_stage(KParams p, int use_flat) {
  constexpr uint32_t NW = RECV_THREADS / 64;
  constexpr uint32_t R = RECV_PER_THREAD;
  __shared__ uint32_t s_ppre[RECV_THREADS];     // entry starts of the block's partitions
  __shared__ uint64_t s_roff[RECV_THREADS];     // list offsets of the block's partitions
  __shared__ uint64_t s_seg[RECV_BATCH];
  __shared__ uint32_t s_epre[RECV_BATCH];
  __shared__ uint32_t s_wsum[NW];
  __shared__ uint64_t s_red[2 * NW];
  __shared__ uint32_t l_pos[SNN_MAX_DELAY];
  const uint32_t tid = threadIdx.x, b = blockIdx.x;
  const uint32_t md = p.D - 1;
  const uint32_t row = p.st->cur_srow;   // counter row
  const uint32_t ppb = (p.P + STAGE_BLOCKS - 1) / STAGE_BLOCKS;
  const uint32_t q0 = min(b * ppb, p.P), q1 = min(q0 + ppb, p.P);
  const uint32_t nq = q1 - q0;
  const uint64_t* lists = use_flat ? p.flat : p.recv;
  const uint32_t* cnts = use_flat ? p.flat_cnt : p.recv_cnt;
  if (tid < SNN_MAX_DELAY) l_pos[tid] = 0;
  uint32_t c = 0;
  if (tid < nq) {
    const uint64_t o = p.recv_off[q0 + tid], o1 = p.recv_off[q0 + tid + 1];
    s_roff[tid] = o;
    c = static_cast<uint32_t>(min(static_cast<uint64_t>(cnts[(q0 + tid) * CNT_STRIDE]), o1 - o));
  }
  uint32_t n_ent;
  s_ppre[tid] = block_excl_scan(c, s_wsum, &n_ent);
  __syncthreads();
  const StageCtx ctx{p.stage + static_cast<uint64_t>(b) * p.stage_cap,
                     static_cast<uint64_t>(STAGE_BLOCKS) * p.stage_cap, p.st->cur_slot, l_pos,
                     s_seg, s_epre, s_wsum};
  uint64_t events = 0;
  for (uint32_t b0 = 0; b0 < n_ent; b0 += RECV_BATCH) {
    const uint32_t nb = min(n_ent - b0, RECV_BATCH);
    uint64_t ent[R];
#pragma unroll
    for (int v = 0; v < R; ++v) {
      const uint32_t e = b0 + min(tid * R + v, nb - 1);
      const uint32_t k = owner_of<STAGE_PARTS / 2>(s_ppre, nq, e);
      ent[v] = lists[s_roff[k] + (e - s_ppre[k])];
    }
    stage_batch<BF16>(p, ctx, ent, nb, events);
  }
  if (tid < md)
    p.stage_cnt[tid * STAGE_BLOCKS + b] =
        static_cast<uint32_t>(min(static_cast<uint64_t>(l_pos[tid]), p.stage_cap));
  add_stat(stat_copy(p, row) + SNN_STAT_REMOTE_EVENTS, events, s_red);
}

__device__ __forceinline__ uint32_t popc_mask(uint32_t m) { return __popc(m); }
__device__ __forceinline__ uint32_t popc_mask(uint64_t m) { return __popcll(m); }
__device__ __forceinline__ uint32_t lowest_bit(uint32_t m) { return __ffs(m) - 1; }
__device__ __forceinline__ uint32_t lowest_bit(uint64_t m) {
  return __ffsll(static_cast<unsigned long long>(m)) - 1;
}

// Mask expansion at the destination node (the bridge's forwarding of
// Sec. IV-B), with or without the staging of the entries (STAGE).  A node's
// messages are split among S = split_of(n_nodes, nblocks) consecutive blocks
// (S = 1 when there are at least as many nodes as blocks: block b then takes
// the nodes b, b + nblocks, ...), so that a shape with few nodes still puts
// every block to work.  A block's messages are loaded EXPAND_PER_THREAD
// consecutive ones per thread; every set bit g of a mask is one receive entry
// (source, pair index of partition G*n + g: the node's destinations are
// consecutive in the source's list, so the pair indices follow the message's
// first one).  Receive-list positions: with S = 1 the block owns the node's
// partitions and counts in LDS; with S > 1 each round's entries are first
// buffered with their partition and rank, then one global atomic per
// partition reserves the round's run in that list.  With STAGE the entries
// also go into an LDS buffer, at positions from a block scan of the masks'
// bit counts, and the buffer is staged per delay (stage_batch) when it is
// full and at the end, without reading the receive lists back; messages
// whose entries do not fit the buffer's free space are taken in the next
// round.
// Block b of nblocks; with STAGE, dyn holds EXPAND_STAGE_LDS bytes of LDS.
// WIDE: groups of more than NARROW_G partitions (masks held in 64 bits,
// otherwise in 32).
__device__ __forceinline__ uint32_t split_of(const KParams& p, uint32_t nblocks) {
  if (p.n_nodes >= nblocks) return 1u;
  const uint32_t s = nblocks / p.n_nodes;
  return p.recv_split ? min(s, p.recv_split) : s;
}

template <bool BF16, bool STAGE, bool WIDE>
__device__ void expand_stage_block(const KParams& p, uint32_t b, uint32_t nblocks, uint64_t* dyn) {
  using MaskT = std::conditional_t<WIDE, uint64_t, uint32_t>;
  constexpr uint32_t NW = RECV_THREADS / 64;
  constexpr uint32_t R = RECV_PER_THREAD;
  constexpr uint32_t EU = EXPAND_PER_THREAD;
  constexpr uint32_t NG = SNN_MAX_GPUS_PER_NODE;
  uint64_t* s_ent = dyn;                                                   // [EXPAND_BUF]
  uint64_t* s_seg = s_ent + EXPAND_BUF;                                    // [RECV_BATCH]
  uint32_t* s_epre = reinterpret_cast<uint32_t*>(s_seg + RECV_BATCH);      // [RECV_BATCH]
  // shared nodes: partition | rank << 8 of each buffered entry of the round,
  // in s_epre (free until the buffer is staged)
  uint32_t* s_gr = s_epre;
  static_assert(RECV_BATCH >= EXPAND_BUF, "the round's ranks fit the staging scratch");
  __shared__ uint32_t s_wsum[NW];
  __shared__ uint64_t s_red[2 * NW];
  __shared__ uint32_t l_pos[SNN_MAX_DELAY];
  __shared__ uint32_t l_cnt[NG], l_run[NG];
  __shared__ uint64_t l_off[NG + 1], l_base[NG];
  __shared__ uint32_t s_taken, s_added;
  const uint32_t tid = threadIdx.x;
  const uint32_t md = p.D - 1;
  const uint32_t row = p.st->cur_srow;   // counter row
  const uint32_t* bcnt = bucket_counts(p, p.st->cur_par);
  if (tid < SNN_MAX_DELAY) l_pos[tid] = 0;
  const StageCtx ctx{p.stage + static_cast<uint64_t>(b) * p.stage_cap,
                     static_cast<uint64_t>(STAGE_BLOCKS) * p.stage_cap, p.st->cur_slot, l_pos,
                     s_seg, s_epre, s_wsum};
  uint64_t events = 0, entries = 0;
  // stages the n buffered entries (uniform n)
  auto stage_buffer = [&](uint32_t n) {
    if constexpr (STAGE) {
      for (uint32_t b0 = 0; b0 < n; b0 += RECV_BATCH) {
        const uint32_t nb = min(n - b0, RECV_BATCH);
        uint64_t ent[R];
#pragma unroll
        for (int v = 0; v < R; ++v) ent[v] = s_ent[b0 + min(tid * R + v, nb - 1)];
        stage_batch<BF16>(p, ctx, ent, nb, events);
      }
    }
  };
  // S blocks per node: block b takes part b mod S of node b / S, then, with
  // S = 1, every nblocks-th node
  const uint32_t S = STAGE ? split_of(p, nblocks) : 1u;
  const bool shared = S > 1;
  const uint32_t n_step = shared ? p.n_nodes : nblocks;   // shared: one node per block
  uint32_t n_buf = 0;   // entries in the buffer (uniform)
  // block-uniform values are kept in scalar registers (readfirstlane): held
  // across the round loop in vector registers they would be spilled
  auto uni = [](uint32_t v) { return __builtin_amdgcn_readfirstlane(v); };
  const uint32_t node0 = uni(b / S), part = uni(b - node0 * S);
  for (uint32_t n = node0; n < p.n_nodes; n += n_step) {
    const uint64_t off = p.bucket_off[n];
    const uint32_t cnt_n = uni(static_cast<uint32_t>(
        min(static_cast<uint64_t>(bcnt[n * CNT_STRIDE]), p.bucket_off[n + 1] - off)));
    // this block's share of the node's messages [m_lo, cnt): S near-equal
    // parts (32-bit arithmetic only: a 64-bit division here spills registers)
    const uint32_t q = uni(cnt_n / S), r = uni(cnt_n - q * S);
    const uint32_t m_lo = uni(q * part + min(part, r));
    const uint32_t cnt = uni(m_lo + q + (part < r ? 1u : 0u));
    const uint32_t gn = uni(min(p.G, p.P - p.G * n));        // partitions of this node
    const MaskT valid = gn == 8 * sizeof(MaskT) ? ~MaskT(0) : (MaskT(1) << gn) - 1;
    __syncthreads();   // the previous node is done with l_run, l_off
    if (tid < NG) l_run[tid] = 0;
    if (tid <= gn) l_off[tid] = p.recv_off[p.G * n + tid];
    for (uint32_t m0 = m_lo; m0 < cnt;) {
      uint64_t w0[EU], w1[EU];
      MaskT mask[EU];
      uint32_t mine = 0;
#pragma unroll
      for (int v = 0; v < EU; ++v) {
        const uint32_t m = m0 + tid * EU + v;
        const uint64_t at = 2 * (off + min(m, cnt - 1));
        w0[v] = p.bucket[at];
        w1[v] = p.bucket[at + 1];
      }
#pragma unroll
      for (int v = 0; v < EU; ++v) {
        const bool in = m0 + tid * EU + v < cnt;
        if (in && (w1[v] & ~static_cast<uint64_t>(valid))) atomicOr(&p.st->error, ERR_ROUTE);
        mask[v] = in ? static_cast<MaskT>(w1[v]) & valid : 0u;
        mine += popc_mask(mask[v]);
      }
      if (tid < NG) l_cnt[tid] = 0;
      if (tid == 0) s_taken = s_added = 0;
      uint32_t total;
      uint32_t at = block_excl_scan(mine, s_wsum, &total);   // ends with the block's view of l_cnt = 0
      const uint32_t room = STAGE ? EXPAND_BUF - n_buf : 0xFFFFFFFFu;
      uint32_t taken = 0, added = 0;
#pragma unroll
      for (int v = 0; v < EU; ++v) {
        const uint32_t pc = popc_mask(mask[v]);
        const bool in = m0 + tid * EU + v < cnt;
        if (in && at + pc <= room) {   // taken (the taken messages are a prefix)
          const uint64_t s = w0[v] & 0xFFFFFFFFull;
          const uint64_t pair = w0[v] >> 32;
          MaskT mm = mask[v];
          uint32_t k = 0;
          while (mm) {
            const uint32_t g = lowest_bit(mm);
            mm &= mm - 1;
            const uint64_t e = s | ((pair + k) << ENTRY_SRC_BITS);
            if constexpr (STAGE) s_ent[n_buf + at + k] = e;
            const uint32_t rk = atomicAdd(&l_cnt[g], 1u);
            if (shared) {
              s_gr[n_buf + at + k] = g | (rk << 8);
            } else {
              const uint64_t pos = l_off[g] + l_run[g] + rk;
              if (pos < l_off[g + 1]) p.recv[pos] = e;
              else atomicOr(&p.st->error, ERR_RECV);
            }
            ++k;
          }
          ++taken;
          added += pc;
        }
        at += pc;
      }
      if (taken) {
        atomicAdd(&s_taken, taken);
        atomicAdd(&s_added, added);
      }
      __syncthreads();
      const uint32_t round_taken = s_taken, round_added = s_added;
      const uint32_t loaded = min(cnt - m0, EU * RECV_THREADS);
      if (shared) {
        // reserve the round's run in each partition's list, then write the
        // buffered entries there
        if (tid < gn && l_cnt[tid])
          l_base[tid] = atomicAdd(p.recv_cnt + (p.G * n + tid) * CNT_STRIDE, l_cnt[tid]);
        __syncthreads();
        for (uint32_t i = tid; i < round_added; i += RECV_THREADS) {
          const uint32_t gr = s_gr[n_buf + i];
          const uint32_t g = gr & 0xFFu;
          const uint64_t pos = l_off[g] + l_base[g] + (gr >> 8);
          if (pos < l_off[g + 1]) p.recv[pos] = s_ent[n_buf + i];
          else atomicOr(&p.st->error, ERR_RECV);
        }
      } else if (tid < NG) {
        l_run[tid] += l_cnt[tid];
      }
      entries += tid == 0 ? round_added : 0u;
      if constexpr (STAGE) n_buf += round_added;
      m0 += round_taken;
      if (round_taken < loaded) {   // the buffer is full: stage it
        __syncthreads();
        stage_buffer(n_buf);
        n_buf = 0;
      }
      __syncthreads();
    }
    if (!shared && tid < gn) p.recv_cnt[(p.G * n + tid) * CNT_STRIDE] = l_run[tid];
  }
  stage_buffer(n_buf);
  if (STAGE && tid < md) {
    const uint32_t c = static_cast<uint32_t>(min(static_cast<uint64_t>(l_pos[tid]), p.stage_cap));
    p.stage_cnt[tid * STAGE_BLOCKS + b] = c;
  }
  uint64_t* sc = stat_copy(p, row);
  add_stats(sc + SNN_STAT_REMOTE_EVENTS, events, sc + SNN_STAT_RECV_ENTRIES, entries, s_red);
}

// Mask expansion alone (the step-by-step path): expansion blocks over the
// nodes, the receive lists as output.
__global__ __launch_bounds__(RECV_THREADS) void k_expand(KParams p) {
  if (p.G > NARROW_G) expand_stage_block<false, false, true>(p, blockIdx.x, gridDim.x, nullptr);
  else expand_stage_block<false, false, false>(p, blockIdx.x, gridDim.x, nullptr);
}

// ---------------------------------------------------------------------------
// deliver: per delay, counting-sort events by tile into private sub-bins

// Block (w, d): the delay-d run of the local segment of fired sources
// w, w + DELIVER_BLOCKS, ..., and the staging queues q = w (mod
// DELIVER_BLOCKS) of delay d.  Every event lands in ring slot (t + d) mod D,
// so the block counting-sorts them by tile in LDS and writes each tile's run
// into sub-bin (slot, tile, d, w).  That sub-bin is written by this block
// only, once per ring cycle, and read by the tile's update D - d steps later:
// positions and counts need no atomics.
// Runs (the source segments in batches of a block's width, then the QPB
// queues) are taken as one flat sequence per batch: one thread per run loads
// its start and length, a block scan concatenates them, and the events are
// taken in rounds of DELIVER_ROUND, GATHER_UNROLL per thread held in
// registers (the owner of an event is found by a power-of-two search).  A
// round is sorted where it stands: each event's rank in its tile comes from
// an LDS counter, a scan of the counts gives the tiles' starts, the events
// are placed in tile order in LDS (8 bytes each), and consecutive threads
// then write consecutive positions of one sub-bin.
// PART: DELIVER_ALL takes the queues after the sources (one kernel per row,
// the queues complete at launch); DELIVER_LOCAL takes the sources only
// (beside the staging, which is still filling the queues) and
// DELIVER_REMOTE the queues only, appended after the counts DELIVER_LOCAL
// published; DELIVER_SPLIT takes the sources, waits for the staging blocks
// of the same launch whose queues it bins (wait_staged), then takes the
// queues, appending to the same runs.
// dyn holds deliver_lds_bytes(n_tiles) bytes.
enum DeliverPart { DELIVER_ALL, DELIVER_LOCAL, DELIVER_REMOTE, DELIVER_SPLIT };
constexpr uint32_t DELIVER_ROUND = GATHER_UNROLL * DELIVER_THREADS;
static_assert(DELIVER_ROUND <= 65536, "window positions fit 16 bits");

// Polls of a wait between blocks of one launch before it gives up with
// ERR_TIMEOUT (each poll sleeps about 128 cycles): every wait ends.
constexpr uint32_t SPIN_LIMIT = 1u << 22;

// The hand-off of the one-launch receive side.  Staging block b publishes
// flag word b (its own 64-byte line) once its queues and counts are stored:
// tag << 4 | the XCD it ran on, the tag being the step counter as this
// launch reads it (at least 1: the update has advanced it), so neither the
// zeroed words of a new handle nor the words of the previous step match.  The
// tag keeps the counter's low 28 bits: a word written by a one-launch receive
// side exactly k * 2^28 steps earlier, with none in between, would match, so
// the host runs such a step's receive side as two launches instead.
__device__ __forceinline__ uint32_t staged_word(const KParams& p, uint32_t xcc) {
  return (static_cast<uint32_t>(p.st->t) << 4) | xcc;
}

// Called by every thread of a staging block once its queues and their
// counts are stored: waits for its own stores to complete (the L1 writes
// through, so they are then in its XCD's L2), then publishes its flag with a
// device-coherent store.
__device__ void signal_staged(const KParams& p) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0)
    __hip_atomic_store(p.sync + SYNC_STRIDE * blockIdx.x, staged_word(p, xcc_id()),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Waits for the staging blocks whose queues delivery block w bins (w, w +
// DELIVER_BLOCKS, ...), checks that each ran on this block's XCD (so that
// its queue stores are in the L2 this block reads through; ERR_XCD where
// not), then drops this CU's L1 copies (buffer_inv sc0: the vector L1 only).
// An agent-scope acquire (buffer_inv sc1) would also invalidate the XCD's
// L2, which then holds the sub-bin runs being written: measured, it made the
// remote part three times slower.  Every thread calls it.
__device__ void wait_staged(const KParams& p, uint32_t w) {
  static_assert(STAGE_BLOCKS % N_XCD == 0 && DELIVER_BLOCKS % N_XCD == 0,
                "a queue's staging and delivery blocks are a multiple of N_XCD apart");
  constexpr uint32_t QPB = STAGE_BLOCKS / DELIVER_BLOCKS;
  static_assert(QPB <= 64, "one lane per queue");
  if (threadIdx.x < QPB) {
    const uint32_t b = w + threadIdx.x * DELIVER_BLOCKS;
    const uint32_t want = staged_word(p, 0) >> 4;
    uint32_t spins = 0, v;
    while (((v = __hip_atomic_load(p.sync + SYNC_STRIDE * b, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT)) >> 4) != (want & 0x0FFFFFFFu)) {
      __builtin_amdgcn_s_sleep(2);
      if (++spins == SPIN_LIMIT) {
        atomicOr(&p.st->error, ERR_TIMEOUT);
        break;
      }
    }
    if ((v & 0xFu) != xcc_id()) atomicOr(&p.st->error, ERR_XCD);
  }
  __syncthreads();
  asm volatile("buffer_inv sc0" ::: "memory");
}

template <DeliverPart PART, bool BF16>
__device__ void deliver_block(const KParams& p, uint32_t w, uint32_t d, uint64_t* dyn) {
  constexpr uint32_t NT = DELIVER_THREADS;
  constexpr uint32_t NW = NT / 64;
  constexpr uint32_t QPB = STAGE_BLOCKS / DELIVER_BLOCKS;                 // queues per block
  static_assert(QPB <= NT, "one queue per thread");
  Event* s_sorted = reinterpret_cast<Event*>(dyn);                        // [DELIVER_ROUND]
  uint32_t* l_cnt = reinterpret_cast<uint32_t*>(s_sorted + DELIVER_ROUND);  // [n_tiles]
  uint32_t* l_run = l_cnt + p.n_tiles;                                    // [n_tiles]
  uint32_t* l_pre = l_run + p.n_tiles;                                    // [n_tiles]
  __shared__ uint64_t s_base[NT];   // first event of each run (synapse or queue index)
  __shared__ uint32_t s_pre[NT];    // run starts in the concatenation
  __shared__ uint32_t s_wsum[NW];
  __shared__ uint64_t s_red[2 * NW];
  const uint32_t tid = threadIdx.x;

  const uint32_t nF = p.st->n_fired;
  uint32_t slot = p.st->cur_slot + d;
  if (slot >= p.D) slot -= p.D;
  const uint32_t row = p.st->cur_srow;   // counter row
  const uint32_t D = p.D;
  constexpr bool WAITS = PART == DELIVER_SPLIT;   // queues staged by this launch
  constexpr bool LOCAL = PART != DELIVER_REMOTE;
  constexpr bool REMOTE = PART != DELIVER_LOCAL;
  // queue lengths, when the queues are complete at launch: loaded with the
  // sub-bin counts below, in the same round trip
  const uint32_t* qcnt = p.stage_cnt + (d - 1) * STAGE_BLOCKS + w + tid * DELIVER_BLOCKS;
  uint32_t qlen = 0;
  if (PART != DELIVER_SPLIT && REMOTE && tid < QPB) qlen = *qcnt;
  for (uint32_t i = tid; i < p.n_tiles; i += NT) {
    l_run[i] = LOCAL ? 0u : p.bin_cnt[subbin(p, slot, i, d, w)];
    l_cnt[i] = 0;
  }
  __syncthreads();
  uint64_t events = 0;
  const uint64_t dw = (d - 1) * DELIVER_BLOCKS + w;

  // sorts the n events of a round (global target tg[v], weight wq[v] of
  // event v * NT + tid, those with on[v]) by tile and writes them out
  auto sort_round = [&](uint32_t n, const uint32_t (&tg)[GATHER_UNROLL],
                        const int32_t (&wq)[GATHER_UNROLL], const bool (&on)[GATHER_UNROLL]) {
    uint32_t rk[GATHER_UNROLL];
#pragma unroll
    for (int v = 0; v < GATHER_UNROLL; ++v)
      rk[v] = on[v] ? atomicAdd(&l_cnt[tile_of(p, tg[v])], 1u) : 0u;
    __syncthreads();
    {
      // exclusive scan of the round's per-tile counts into l_pre
      const uint32_t per = (p.n_tiles + NT - 1) / NT;
      const uint32_t i0 = min(tid * per, p.n_tiles), i1 = min(i0 + per, p.n_tiles);
      uint32_t sum = 0;
      for (uint32_t i = i0; i < i1; ++i) sum += l_cnt[i];
      uint32_t tot;
      uint32_t ex = block_excl_scan(sum, s_wsum, &tot);
      for (uint32_t i = i0; i < i1; ++i) {
        l_pre[i] = ex;
        ex += l_cnt[i];
      }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < GATHER_UNROLL; ++v)
      if (on[v]) s_sorted[l_pre[tile_of(p, tg[v])] + rk[v]] = Event{tg[v], wq[v]};
    __syncthreads();
    for (uint32_t j = tid; j < n; j += NT) {
      const Event ev = s_sorted[j];
      const uint32_t tile = tile_of(p, ev.tgt);
      const uint64_t pos = static_cast<uint64_t>(l_run[tile]) + (j - l_pre[tile]);
      if (pos < p.bin_cap)
        p.bins[bin_data(p, slot, tile, static_cast<uint32_t>(dw)) + pos] =
            Event{ev.tgt - tile * p.tile, ev.wq};
      else
        ring_fallback(p, slot, ev.tgt, ev.wq);
    }
    __syncthreads();
    for (uint32_t i = tid; i < p.n_tiles; i += NT) {
      l_run[i] += l_cnt[i];
      l_cnt[i] = 0;
    }
    __syncthreads();
  };

  // the events of nseg runs (s_base, len per thread), QUEUE: queue runs of
  // staged events, else synapse runs of the CSR
  auto take_runs = [&](uint32_t nseg, uint32_t len, auto queue_tag) {
    constexpr bool QUEUE = decltype(queue_tag)::value;
    const Event* q0 = p.stage + (static_cast<uint64_t>(d - 1) * STAGE_BLOCKS + w) * p.stage_cap;
    uint32_t tot;
    const uint32_t ex = block_excl_scan(len, s_wsum, &tot);
    s_pre[tid] = ex;
    __syncthreads();
    for (uint32_t r0 = 0; r0 < tot; r0 += DELIVER_ROUND) {
      const uint32_t n = min(tot - r0, DELIVER_ROUND);
      uint32_t tg[GATHER_UNROLL];
      int32_t wq[GATHER_UNROLL];
      bool on[GATHER_UNROLL];
#pragma unroll
      for (int v = 0; v < GATHER_UNROLL; ++v) {
        const uint32_t i = v * NT + tid;
        on[v] = i < n;
        const uint32_t e = r0 + min(i, n - 1);
        const uint32_t k = owner_of<NT / 2>(s_pre, nseg, e);
        const uint64_t x = s_base[k] + (e - s_pre[k]);
        if constexpr (QUEUE) {
          const Event ev = q0[x];
          tg[v] = ev.tgt;
          wq[v] = ev.wq;
        } else {
          tg[v] = p.tgt_delay[x] & 0x07FFFFFFu;
          wq[v] = quantize_w(p, load_weight<BF16>(p, x));
        }
      }
      sort_round(n, tg, wq, on);
    }
    __syncthreads();   // s_pre, s_base are rewritten by the next batch
  };

  // the own-partition synapses of delay d of this block's fired sources
  // (w + m * DELIVER_BLOCKS), NT sources per batch
  const uint32_t M = LOCAL && nF > w ? (nF - w + DELIVER_BLOCKS - 1) / DELIVER_BLOCKS : 0;
  for (uint32_t m0 = 0; m0 < M; m0 += NT) {
    const uint32_t nsrc = min(M - m0, NT);
    uint32_t len = 0;
    if (tid < nsrc) {
      const uint32_t s = p.fired[w + (m0 + tid) * DELIVER_BLOCKS];
      const uint64_t o = static_cast<uint64_t>(s) * D;
      const uint32_t a = p.delay_off[o + d - 1], z = p.delay_off[o + d];
      s_base[tid] = static_cast<uint64_t>(p.row_ptr[s]) + a;
      len = z - a;
      events += len;
    }
    take_runs(nsrc, len, std::false_type{});
  }
  if constexpr (WAITS) wait_staged(p, w);
  // the staged remote synapses of delay d: queues w, w + DELIVER_BLOCKS, ...
  if constexpr (REMOTE) {
    if (tid < QPB) {
      s_base[tid] = static_cast<uint64_t>(tid) * DELIVER_BLOCKS * p.stage_cap;
      if (PART == DELIVER_SPLIT) qlen = *qcnt;
    }
    take_runs(QPB, qlen, std::true_type{});
  }

  // publish this block's counts for slot `slot`, every tile (zeros included)
  for (uint32_t i = tid; i < p.n_tiles; i += NT)
    p.bin_cnt[subbin(p, slot, i, d, w)] =
        static_cast<uint32_t>(min(static_cast<uint64_t>(l_run[i]), p.bin_cap));
  if constexpr (LOCAL) add_stat(stat_copy(p, row) + SNN_STAT_LOCAL_EVENTS, events, s_red);
}

template <bool BF16>
__global__ __launch_bounds__(DELIVER_THREADS) void k_deliver(KParams p) {
  extern __shared__ uint64_t lds_u64[];
  deliver_block<DELIVER_ALL, BF16>(p, blockIdx.x, blockIdx.y + 1, lds_u64);
}

// The staged remote synapses of (w, d) = (blockIdx.x, blockIdx.y + 1), after
// k_recv_local delivered the local ones.
template <bool BF16>
__global__ __launch_bounds__(DELIVER_THREADS) void k_deliver_remote(KParams p) {
  extern __shared__ uint64_t lds_u64[];
  deliver_block<DELIVER_REMOTE, BF16>(p, blockIdx.x, blockIdx.y + 1, lds_u64);
}

// Expansion and staging beside the own-partition delivery: two independent
// jobs in one launch, so that they overlap (block layout as k_recv_deliver);
// the staged queues are binned by k_deliver_remote after it.
template <bool BF16, bool WIDE>
__global__ __launch_bounds__(RECV_THREADS) __attribute__((amdgpu_waves_per_eu(6)))
void k_recv_local(KParams p) {
  extern __shared__ uint64_t lds_u64[];
  if (blockIdx.x < STAGE_BLOCKS) {
    expand_stage_block<BF16, true, WIDE>(p, blockIdx.x, STAGE_BLOCKS, lds_u64);
  } else {
    const uint32_t i = blockIdx.x - STAGE_BLOCKS;
    deliver_block<DELIVER_LOCAL, BF16>(p, i % DELIVER_BLOCKS, i / DELIVER_BLOCKS + 1, lds_u64);
  }
}

// The receive side and the delivery of a step in one launch: blocks
// [0, STAGE_BLOCKS) expand and stage the two-level messages
// (expand_stage_block) and publish their flags when their queues are
// stored; the rest (block STAGE_BLOCKS + i takes (w, d) =
// (i mod DELIVER_BLOCKS, i / DELIVER_BLOCKS + 1)) deliver the fired sources'
// local synapses meanwhile (they need only the fired list), wait for the
// staging blocks, and bin the staged remote synapses.  Only higher-numbered
// blocks wait, for lower-numbered ones, which are dispatched first.  Three
// blocks of 8 waves per CU (6 waves per SIMD, at most 80 VGPRs).
static_assert(RECV_THREADS == DELIVER_THREADS, "one block size for both jobs");
template <bool BF16, bool WIDE>
__global__ __launch_bounds__(RECV_THREADS) __attribute__((amdgpu_waves_per_eu(6)))
void k_recv_deliver(KParams p) {
  extern __shared__ uint64_t lds_u64[];
  if (blockIdx.x < STAGE_BLOCKS) {
    expand_stage_block<BF16, true, WIDE>(p, blockIdx.x, STAGE_BLOCKS, lds_u64);
    signal_staged(p);
  } else {
    const uint32_t i = blockIdx.x - STAGE_BLOCKS;
    deliver_block<DELIVER_SPLIT, BF16>(p, i % DELIVER_BLOCKS, i / DELIVER_BLOCKS + 1, lds_u64);
  }
}

// Writes the input scheduled for the coming steps into the dense ring p.ring
// (binary32, slot-major): for every slot and neuron, the pending fixed-point
// events of its bins plus its overflow-ring sum, rounded as the update will
// round them.  Nothing is moved or cleared, so the simulation continues
// unchanged.  Grid: x = tile, y = slot.  Bins are not cleared when consumed,
// so only some are pending: slot s is consumed k steps from now
// (k = (s - next slot) mod D), and its bin of delay d has been written for
// that step only if d > k (it is written at step s - d); the others still
// hold input already consumed.
__global__ __launch_bounds__(256) void k_flush(KParams p) {
  __shared__ int32_t s_acc[TILE_MAX];
  const uint32_t tile = blockIdx.x, slot = blockIdx.y;
  const uint32_t next = p.st->slot;
  const uint32_t ahead = slot >= next ? slot - next : slot + p.D - next;
  const uint32_t md = p.D - 1;
  const uint32_t blk0 = tile * p.tile;
  const uint32_t nt = min(p.tile, p.N - blk0);
  const uint64_t row = static_cast<uint64_t>(slot) * p.ring_stride + blk0;
  for (uint32_t i = threadIdx.x; i < p.tile; i += 256) s_acc[i] = i < nt ? p.ovf[row + i] : 0;
  __syncthreads();
  for (uint32_t d = ahead + 1; d <= md; ++d) {
    for (uint32_t w = 0; w < DELIVER_BLOCKS; ++w) {
      const uint32_t c = min(p.bin_cnt[subbin(p, slot, tile, d, w)],
                             static_cast<uint32_t>(p.bin_cap));
      const Event* ev = p.bins + bin_data(p, slot, tile, (d - 1) * DELIVER_BLOCKS + w);
      for (uint32_t e = threadIdx.x; e < c; e += 256) atomicAdd(&s_acc[ev[e].tgt], ev[e].wq);
    }
  }
  __syncthreads();
  const float wq_inv = static_cast<float>(p.wq_inv);
  for (uint32_t i = threadIdx.x; i < nt; i += 256)
    p.ring[row + i] = __fmul_rn(static_cast<float>(s_acc[i]), wq_inv);
}

// Set-up kernels of the allocation-free entry point (snn_create_static),
// which writes no memset or host-to-device copy into the stream.

// Zeroes n 32-bit words at dst.
__global__ __launch_bounds__(256) void k_zero_words(uint32_t* dst, uint64_t n) {
  const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
  for (uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
    dst[i] = 0u;
}

// The Poisson inversion lookup (layout in snn_internal.h) from the
// thresholds p.thr: entry b covers the draws [lo, hi] = [b << POIS_LUT_SHIFT,
// lo + 2^POIS_LUT_SHIFT - 1]; no threshold in (lo, hi] fixes k, exactly one
// is resolved by one comparison in the update.
__global__ __launch_bounds__(256) void k_pois_lut(KParams p, uint8_t* lut) {
  const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= POIS_LUT_SIZE) return;
  const uint64_t lo = static_cast<uint64_t>(b) << POIS_LUT_SHIFT;
  const uint64_t hi = lo + (uint64_t(1) << POIS_LUT_SHIFT) - 1;
  uint32_t k_lo = 0, k_hi = 0;
  for (int j = 0; j < 15; ++j) {
    k_lo += p.thr[j] <= lo ? 1u : 0u;
    k_hi += p.thr[j] <= hi ? 1u : 0u;
  }
  lut[b] = k_hi == k_lo ? static_cast<uint8_t>(k_lo)
         : k_hi == k_lo + 1 ? static_cast<uint8_t>(16 + k_lo) : POIS_LUT_SLOW;
}

// ---------------------------------------------------------------------------
// launchers

uint32_t tile_size(uint32_t n, uint32_t requested) {
  if (requested) return requested;
  const uint32_t per = (n + TILE_MIN_COUNT - 1) / TILE_MIN_COUNT;
  const uint32_t t = (per + TILE_ALIGN - 1) / TILE_ALIGN * TILE_ALIGN;
  return std::min(std::max(t, TILE_MIN_DEFAULT), TILE_MAX);
}

void tile_divider(uint32_t t, uint32_t* magic, uint32_t* shift) {
  // c = ceil(log2 t); magic = ceil(2^(31 + c) / t) < 2^32.  For x < 2^27 the
  // error of x * magic / 2^(31 + c) against x / t is below 2^27 / 2^(31 + c)
  // <= 1 / (16 t), too small to carry x / t past the next integer.
  uint32_t c = 0;
  while ((1u << c) < t) ++c;
  const uint64_t k = uint64_t(1) << (31 + c);
  *magic = static_cast<uint32_t>((k + t - 1) / t);
  *shift = c - 1;
}

// Optional timing marks: when marks is non-null, events marks[2k] and
// marks[2k + 1] are recorded on the stream around each launch of kernel kind
// k (SNN_KERNEL_*).
static inline void mark(hipEvent_t* marks, int kind, int end, hipStream_t s) {
  if (marks) (void)hipEventRecord(marks[2 * kind + end], s);
}

bool fused_route_ok(const KParams& p) { return p.n_nodes <= FUSED_MAX_NODES && p.G <= NARROW_G; }

hipError_t launch_update(const KParams& p, hipStream_t s, hipEvent_t* marks, bool route) {
  mark(marks, SNN_KERNEL_UPDATE, 0, s);
  const uint32_t tiles = p.tile_end - p.tile0;
  const bool persist = p.update_blocks && p.update_blocks < tiles && p.tile0 == 0 &&
                       p.tile_end == p.n_tiles;
  const uint32_t grid = persist ? p.update_blocks : tiles;
  const bool r = route && fused_route_ok(p);
  void (*kern)(KParams) = persist ? (r ? k_update<true, true> : k_update<false, true>)
                                  : (r ? k_update<true, false> : k_update<false, false>);
  hipLaunchKernelGGL(kern, dim3(grid), dim3(UPDATE_THREADS), 0, s, p);
  mark(marks, SNN_KERNEL_UPDATE, 1, s);
  return hipGetLastError();
}

static size_t route_kernel_lds_bytes(const KParams& p) {
  return route_lds_bytes(ROUTE_THREADS, ROUTE_STAGE, p.n_nodes, p.G > NARROW_G);
}

hipError_t launch_route(const KParams& p, int mode, hipStream_t s, hipEvent_t* marks,
                        bool routed, bool defer_expand) {
  if (mode == SNN_ROUTE_TWO_LEVEL || mode == SNN_ROUTE_BOTH) {
    if (!routed) {
      mark(marks, SNN_KERNEL_ROUTE_TWO_LEVEL, 0, s);
      if (p.n_nodes <= ROUTE_MAX_NODES_LDS)
        hipLaunchKernelGGL(p.G > NARROW_G ? k_route_two_level<true> : k_route_two_level<false>,
                           dim3(ROUTE_BLOCKS), dim3(ROUTE_THREADS),
                           route_kernel_lds_bytes(p), s, p);
      else
        hipLaunchKernelGGL(k_route_two_level_direct, dim3(1024), dim3(ROUTE_THREADS), 0, s, p);
      mark(marks, SNN_KERNEL_ROUTE_TWO_LEVEL, 1, s);
    }
    if (!defer_expand) {
      mark(marks, SNN_KERNEL_EXPAND, 0, s);
      hipLaunchKernelGGL(k_expand, dim3(std::min(p.n_nodes, STAGE_BLOCKS)), dim3(RECV_THREADS), 0,
                         s, p);
      mark(marks, SNN_KERNEL_EXPAND, 1, s);
    }
  }
  if (mode == SNN_ROUTE_FLAT || mode == SNN_ROUTE_BOTH) {
    mark(marks, SNN_KERNEL_ROUTE_FLAT, 0, s);
    hipLaunchKernelGGL(k_route_flat, dim3(1024), dim3(ROUTE_THREADS), 0, s, p);
    mark(marks, SNN_KERNEL_ROUTE_FLAT, 1, s);
  }
  return hipGetLastError();
}

// LDS of a deliver block: a round of events in tile order and three
// counters per tile.
static size_t deliver_lds_bytes(uint32_t n_tiles) {
  return DELIVER_ROUND * sizeof(Event) + 3ull * n_tiles * sizeof(uint32_t);
}

// Expansion and staging: the entry buffer, and per batch each entry's
// segment start and its remaining synapses' start.
constexpr size_t EXPAND_STAGE_LDS =
    EXPAND_BUF * sizeof(uint64_t) + RECV_BATCH * (sizeof(uint64_t) + sizeof(uint32_t));

static size_t recv_deliver_lds_bytes(const KParams& p) {
  return std::max(EXPAND_STAGE_LDS, deliver_lds_bytes(p.n_tiles));
}

template <bool BF16>
static void launch_deliver_t(const KParams& p, int mode, hipStream_t s, hipEvent_t* marks,
                             bool fused_expand) {
  if (fused_expand && mode != SNN_ROUTE_FLAT) {
    const dim3 grid(STAGE_BLOCKS + DELIVER_BLOCKS * (p.D - 1));
    mark(marks, SNN_KERNEL_RECV_STAGE, 0, s);
    if (p.recv_merged) {
      void (*kern)(KParams) =
          p.G > NARROW_G ? k_recv_deliver<BF16, true> : k_recv_deliver<BF16, false>;
      hipLaunchKernelGGL(kern, grid, dim3(RECV_THREADS), recv_deliver_lds_bytes(p), s, p);
      mark(marks, SNN_KERNEL_RECV_STAGE, 1, s);
      return;
    }
    void (*kern)(KParams) = p.G > NARROW_G ? k_recv_local<BF16, true> : k_recv_local<BF16, false>;
    hipLaunchKernelGGL(kern, grid, dim3(RECV_THREADS), recv_deliver_lds_bytes(p), s, p);
    mark(marks, SNN_KERNEL_RECV_STAGE, 1, s);
    mark(marks, SNN_KERNEL_DELIVER, 0, s);
    hipLaunchKernelGGL(k_deliver_remote<BF16>, dim3(DELIVER_BLOCKS, p.D - 1),
                       dim3(DELIVER_THREADS), deliver_lds_bytes(p.n_tiles), s, p);
    mark(marks, SNN_KERNEL_DELIVER, 1, s);
    return;
  }
  mark(marks, SNN_KERNEL_RECV_STAGE, 0, s);
  hipLaunchKernelGGL(k_recv_stage<BF16>, dim3(STAGE_BLOCKS), dim3(RECV_THREADS), 0, s, p,
                     mode == SNN_ROUTE_FLAT ? 1 : 0);
  mark(marks, SNN_KERNEL_RECV_STAGE, 1, s);
  mark(marks, SNN_KERNEL_DELIVER, 0, s);
  hipLaunchKernelGGL(k_deliver<BF16>, dim3(DELIVER_BLOCKS, p.D - 1), dim3(DELIVER_THREADS),
                     deliver_lds_bytes(p.n_tiles), s, p);
  mark(marks, SNN_KERNEL_DELIVER, 1, s);
}

hipError_t launch_deliver(const KParams& p, int mode, hipStream_t s, hipEvent_t* marks,
                          bool fused_expand) {
  if (p.bf16) launch_deliver_t<true>(p, mode, s, marks, fused_expand);
  else launch_deliver_t<false>(p, mode, s, marks, fused_expand);
  return hipGetLastError();
}

// Static plus dynamic LDS of kernel f fits the device, and f may use dyn bytes.
static hipError_t allow_lds(const void* f, size_t dyn, int lds_max) {
  hipFuncAttributes fa{};
  hipError_t e = hipFuncGetAttributes(&fa, f);
  if (e != hipSuccess) return e;
  if (int64_t(fa.sharedSizeBytes + dyn) > lds_max) return hipErrorInvalidConfiguration;
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(dyn));
}

hipError_t prepare_kernels(KParams& p) {
  int dev = 0, lds_max = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
  if (e != hipSuccess) return e;
  // the deliver kernels' per-tile counters must leave room for a round
  const size_t dl = deliver_lds_bytes(p.n_tiles), rl = recv_deliver_lds_bytes(p);
  const std::pair<const void*, size_t> kernels[] = {
      {reinterpret_cast<const void*>(&k_deliver<false>), dl},
      {reinterpret_cast<const void*>(&k_deliver<true>), dl},
      {reinterpret_cast<const void*>(&k_deliver_remote<false>), dl},
      {reinterpret_cast<const void*>(&k_deliver_remote<true>), dl},
      {reinterpret_cast<const void*>(&k_recv_local<false, false>), rl},
      {reinterpret_cast<const void*>(&k_recv_local<true, false>), rl},
      {reinterpret_cast<const void*>(&k_recv_local<false, true>), rl},
      {reinterpret_cast<const void*>(&k_recv_local<true, true>), rl},
      {reinterpret_cast<const void*>(&k_recv_deliver<false, false>), rl},
      {reinterpret_cast<const void*>(&k_recv_deliver<true, false>), rl},
      {reinterpret_cast<const void*>(&k_recv_deliver<false, true>), rl},
      {reinterpret_cast<const void*>(&k_recv_deliver<true, true>), rl},
      {reinterpret_cast<const void*>(&k_route_two_level<false>), route_kernel_lds_bytes(p)},
      {reinterpret_cast<const void*>(&k_route_two_level<true>), route_kernel_lds_bytes(p)},
  };
  for (const auto& k : kernels) {
    e = allow_lds(k.first, k.second, lds_max);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_zero(void* dst, uint64_t bytes, hipStream_t s) {
  const uint64_t words = bytes / 4;
  const uint32_t blocks = static_cast<uint32_t>(std::min<uint64_t>((words + 255) / 256, 4096));
  if (blocks) hipLaunchKernelGGL(k_zero_words, dim3(blocks), dim3(256), 0, s,
                                 static_cast<uint32_t*>(dst), words);
  return hipGetLastError();
}

hipError_t launch_pois_lut(const KParams& p, uint8_t* lut, hipStream_t s) {
  hipLaunchKernelGGL(k_pois_lut, dim3(POIS_LUT_SIZE / 256), dim3(256), 0, s, p, lut);
  return hipGetLastError();
}

hipError_t launch_flush(const KParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_flush, dim3(p.n_tiles, p.D), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace snn
