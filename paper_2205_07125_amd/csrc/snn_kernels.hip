// snn_kernels.hip — the per-step kernels for gfx950 (wave64, CDNA4).
//
//   update       one block per tile of TILE neurons: sums the tile's arriving
//                synaptic events into LDS from its bins, runs the LIF update
//                and threshold, compacts fired ids in ascending order (wave
//                ballots, block scan, decoupled look-back across tiles)
//   route        two-level: one (source, node mask) message per destination
//                node into per-node buckets (Sec. IV-B), then mask expansion
//                into per-partition receive lists (the bridge's forwarding);
//                flat: one receive entry per destination partition
//   recv_stage   receive side: each entry's synapses for its partition,
//                staged per delay in per-block queues
//   deliver      per delay: the own-partition synapses of every fired source
//                plus the staged remote ones, counting-sorted by tile in LDS
//                and written as runs into per-(slot, tile, delay, block) bins
//
// Global atomics run at roughly 20 G/s on random addresses and serialise on
// hot counters, so every scatter goes through LDS first: reservations are one
// atomic per round and counter (routing), or none at all (the bins are private
// per writer and written once per ring cycle).  The dense delay ring is only a
// fallback for events that do not fit their bin; its tiles are read when
// flagged.  The work is sparse gather/scatter: no dense contraction, no MFMA.
// Compiled with -ffp-contract=off: the membrane update rounds after every
// operation, exactly as specified.
#include "snn_internal.h"

namespace snn {

// ---------------------------------------------------------------------------
// helpers

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of the
// multiply-xor S-box with a Weyl-bumped key.
__device__ __forceinline__ uint4 philox4x32_10(uint32_t c0, uint32_t c1, uint32_t c2,
                                               uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(0xD2511F53u, c0), lo0 = 0xD2511F53u * c0;
    const uint32_t hi1 = __umulhi(0xCD9E8D57u, c2), lo1 = 0xCD9E8D57u * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0;
    const uint32_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
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

__device__ __forceinline__ float load_weight(const KParams& p, uint64_t e) {
  if (p.bf16) {
    const uint16_t b = static_cast<const uint16_t*>(p.weight)[e];
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
  }
  return static_cast<const float*>(p.weight)[e];
}

// Adds a per-thread counter into a global u64 with one atomic per wave.
__device__ __forceinline__ void add_stat(uint64_t* dst, uint64_t v) {
  v = wave_sum64(v);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(reinterpret_cast<unsigned long long*>(dst), v);
}

// An event that does not fit its bin goes to the dense ring; the tile is
// flagged so the update kernel reads that slice of the ring.
__device__ void ring_fallback(const KParams& p, uint32_t slot, uint32_t tgt, float w) {
  unsafeAtomicAdd(p.ring + slot * p.ring_stride + tgt, w);
  p.dirty[slot * p.n_tiles + (tgt >> TILE_SHIFT)] = 1u;
  atomicAdd(reinterpret_cast<unsigned long long*>(&p.st->ring_events), 1ull);
}

// Sub-bin (slot, tile, delay d in 1..max_delay, deliver block w) of events.
__device__ __forceinline__ uint64_t subbin(const KParams& p, uint32_t slot, uint32_t tile,
                                           uint32_t d, uint32_t w) {
  const uint32_t md = p.D - 1;
  return ((static_cast<uint64_t>(slot) * p.n_tiles + tile) * md + (d - 1)) * DELIVER_BLOCKS + w;
}

// ---------------------------------------------------------------------------
// update: arriving input, neuron update, threshold, ascending compaction

// Look-back word: [63:34] step tag, [33:32] status, [31:0] count.
constexpr uint32_t LB_AGG = 1u, LB_INCL = 2u;

__device__ __forceinline__ uint64_t lb_pack(uint32_t tag, uint32_t status, uint32_t v) {
  return (static_cast<uint64_t>(tag) << 34) | (static_cast<uint64_t>(status) << 32) | v;
}

// Wave 0 of block b: publishes the block's count, walks back over the
// predecessors 64 at a time until an inclusive prefix closes the window, and
// publishes the inclusive prefix.  Returns the exclusive prefix.
// The 64-bit word carries tag, status and count together and nothing else
// is read through it, so relaxed device-scope atomics suffice: acquire or
// release would add an L2 invalidate or write-back to every poll.
__device__ uint32_t lookback_exclusive(uint64_t* lb, uint32_t b, uint32_t agg, uint32_t tag) {
  const int lane = threadIdx.x & 63;
  if (b == 0) {
    if (lane == 0)
      __hip_atomic_store(lb, lb_pack(tag, LB_INCL, agg), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0)
    __hip_atomic_store(lb + b, lb_pack(tag, LB_AGG, agg), __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
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

// One block per tile.  Thread tid owns 16 neurons as 4 quads: quad q covers
// tile neurons q*4*UPDATE_THREADS + 4*tid .. +3, so every load and store
// instruction of a wave touches one contiguous 1 KiB span.  Ids are ordered
// quad-major across the block, which the compaction follows.
__global__ __launch_bounds__(UPDATE_THREADS) void k_update(KParams p) {
  constexpr int NQ = UPDATE_NPT / 4;
  constexpr int NW = UPDATE_THREADS / 64;
  __shared__ float s_syn[TILE];
  __shared__ uint32_t s_cnt[NQ][NW];
  __shared__ uint32_t s_excl;
  __shared__ uint32_t s_dirty;

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
  const uint32_t phase = rd32(&st->phase);
  const uint32_t tag = rd32(&st->tag) + 1u;
  const uint64_t log_head =
      (static_cast<uint64_t>(rd32(reinterpret_cast<const uint32_t*>(&st->log_head) + 1)) << 32) |
      rd32(reinterpret_cast<const uint32_t*>(&st->log_head));
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t tile = blockIdx.x;
  const uint32_t blk0 = tile * TILE;

  // Per-step counters of the routing kernels that follow.
  if (blockIdx.x == 0) {
    for (uint32_t i = tid; i < p.n_nodes; i += UPDATE_THREADS) p.bucket_cnt[i * CNT_STRIDE] = 0;
    for (uint32_t i = tid; i < p.P; i += UPDATE_THREADS) {
      p.recv_cnt[i * CNT_STRIDE] = 0;
      p.flat_cnt[i * CNT_STRIDE] = 0;
    }
    if (tid >= 1 && tid < SNN_NSTAT) p.stats[static_cast<uint64_t>(row) * SNN_NSTAT + tid] = 0;
  }
  for (uint32_t i = tid; i < TILE; i += UPDATE_THREADS) s_syn[i] = 0.f;
  if (tid == 0) s_dirty = p.dirty[slot * p.n_tiles + tile];
  __syncthreads();

  // Arriving input of step t: the sub-bins (slot, tile, d, w) written d steps
  // ago by deliver block w; one wave per sub-bin.
  const uint32_t md = p.D - 1;
  const uint32_t n_sub = md * DELIVER_BLOCKS;
  const uint64_t sb0 = subbin(p, slot, tile, 1, 0);
  for (uint32_t k = wave; k < n_sub; k += NW) {
    const uint64_t sb = sb0 + k;
    const uint32_t c = min(p.bin_cnt[sb], static_cast<uint32_t>(p.bin_cap));
    const Event* ev = p.bins + sb * p.bin_cap;
    for (uint32_t e = lane; e < c; e += 64) {
      const Event x = ev[e];
      atomicAdd(&s_syn[x.tgt], x.w);
    }
  }
  __syncthreads();
  float* ring_slot = p.ring + static_cast<uint64_t>(slot) * p.ring_stride;
  if (s_dirty) {
    // events that did not fit their bins: this tile's slice of the ring slot
    for (uint32_t i = tid; i < TILE; i += UPDATE_THREADS) {
      if (blk0 + i < p.N) {
        s_syn[i] += ring_slot[blk0 + i];
        ring_slot[blk0 + i] = 0.f;
      }
    }
    __syncthreads();
    if (tid == 0) p.dirty[slot * p.n_tiles + tile] = 0u;
  }

  uint32_t thr_raster = 0;
  if (p.forced) thr_raster = phase < p.raster_on ? p.raster_on_thr : p.raster_off_thr;

  uint32_t fire_bits = 0;   // bit 4q + k: neuron k of quad q fired
  // Quads one at a time (not unrolled): keeps the kernel near 64 VGPRs so two
  // 1024-thread blocks fit a CU and every tile of the network is resident.
#pragma unroll 1
  for (int q = 0; q < NQ; ++q) {
    const uint32_t l0 = q * (4 * UPDATE_THREADS) + 4 * tid;
    const uint32_t i0 = blk0 + l0;
    // Philox counter word 0 is i0 / 4: one call serves the quad's 4 neurons.
    const uint4 rnd = philox4x32_10(i0 >> 2, t32, STREAM_POISSON, 0u, p.seed_lo, p.seed_hi);
    uint4 rnd2 = make_uint4(0, 0, 0, 0);
    if (p.forced) rnd2 = philox4x32_10(i0 >> 2, t32, STREAM_RASTER, 0u, p.seed_lo, p.seed_hi);
    const uint32_t r1[4] = {rnd.x, rnd.y, rnd.z, rnd.w};
    const uint32_t r2[4] = {rnd2.x, rnd2.y, rnd2.z, rnd2.w};
    float uu[4] = {0.f, 0.f, 0.f, 0.f};
    uint32_t rf[4] = {0, 0, 0, 0};
    const bool full = i0 + 4 <= p.N;
    if (full) {
      const float4 u4 = *reinterpret_cast<const float4*>(p.u + i0);
      const uint32_t r4 = *reinterpret_cast<const uint32_t*>(p.ref + i0);
      uu[0] = u4.x; uu[1] = u4.y; uu[2] = u4.z; uu[3] = u4.w;
#pragma unroll
      for (int k = 0; k < 4; ++k) rf[k] = (r4 >> (8 * k)) & 0xFFu;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i0 + k < p.N) {
          uu[k] = p.u[i0 + k];
          rf[k] = p.ref[i0 + k];
        }
    }
    const float4 syn4 = *reinterpret_cast<const float4*>(&s_syn[l0]);
    const float syn[4] = {syn4.x, syn4.y, syn4.z, syn4.w};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t kk = 0;
#pragma unroll
      for (int j = 0; j < 15; ++j) kk += p.thr[j] <= r1[k] ? 1u : 0u;
      const float ext = __fmul_rn(static_cast<float>(kk), p.w_ext);
      const bool integrating = rf[k] == 0;
      if (!integrating) {
        rf[k] -= 1;
      } else {
        const float I = __fadd_rn(syn[k], ext);
        const float v = __fmul_rn(uu[k], p.alpha);
        uu[k] = __fadd_rn(v, I);
      }
      bool s = p.forced ? (r2[k] < thr_raster) : (integrating && uu[k] >= p.theta);
      s = s && (i0 + k < p.N);
      if (s) {
        uu[k] = p.u_reset;
        rf[k] = p.n_ref;
      }
      fire_bits |= static_cast<uint32_t>(s) << (4 * q + k);
    }
    if (full) {
      *reinterpret_cast<float4*>(p.u + i0) = make_float4(uu[0], uu[1], uu[2], uu[3]);
      *reinterpret_cast<uint32_t*>(p.ref + i0) =
          rf[0] | (rf[1] << 8) | (rf[2] << 16) | (rf[3] << 24);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i0 + k < p.N) {
          p.u[i0 + k] = uu[k];
          p.ref[i0 + k] = static_cast<uint8_t>(rf[k]);
        }
    }
  }

  // Compaction.  Within quad q, ids ascend with (wave, lane, k); across
  // quads, quad q of every wave precedes quad q + 1.  The rank of a fired id
  // is: fired ids of earlier quads (whole block) + of earlier waves in this
  // quad + of lower lanes in this wave and quad (4 ballots) + earlier k.
  const uint64_t lt = (1ull << lane) - 1ull;
  uint32_t lane_pre[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const uint64_t b = __ballot((fire_bits >> (4 * q + k)) & 1u);
      pre += __popcll(b & lt);
      tot += __popcll(b);
    }
    lane_pre[q] = pre;
    if (lane == 0) s_cnt[q][wave] = tot;
  }
  __syncthreads();
  uint32_t block_tot = 0;
  uint32_t quad_off[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    uint32_t before_wave = 0, quad_tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
      before_wave += w < static_cast<int>(wave) ? s_cnt[q][w] : 0u;
      quad_tot += s_cnt[q][w];
    }
    quad_off[q] = block_tot + before_wave + lane_pre[q];
    block_tot += quad_tot;
  }
  if (wave == 0) {
    const uint32_t excl = lookback_exclusive(p.lookback, blockIdx.x, block_tot, tag);
    if (lane == 0) s_excl = excl;
  }
  __syncthreads();
  if (fire_bits) {
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      uint32_t pos = s_excl + quad_off[q];
      const uint32_t i0 = blk0 + q * (4 * UPDATE_THREADS) + 4 * tid;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if ((fire_bits >> (4 * q + k)) & 1u) {
          p.fired[pos] = i0 + k;
          if (p.log_cap) {
            uint64_t at = log_head + pos;
            if (at >= p.log_cap) at %= p.log_cap;
            p.log[at] = i0 + k;
          }
          ++pos;
        }
    }
  }

  // The last block holds the step total once its look-back is done; every
  // other block has read t and log_total by then (they published first).
  if (blockIdx.x == gridDim.x - 1 && tid == 0) {
    DevState* w = p.st;
    const uint32_t n = s_excl + block_tot;
    const uint64_t log_base = w->log_total;
    w->n_fired = n;
    p.stats[static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_SPIKES] = n;
    p.log_off[row] = log_base;
    if (p.log_cap && n > p.log_cap) atomicOr(&w->error, ERR_LOG);
    w->log_total = log_base + n;
    if (p.log_cap) w->log_head = (w->log_head + n) % p.log_cap;
    w->cur_slot = slot;
    w->cur_row = row;
    w->slot = slot + 1 == p.D ? 0u : slot + 1;
    w->row = row + 1 == p.log_steps ? 0u : row + 1;
    w->phase = phase + 1 == p.raster_period ? 0u : phase + 1;
    w->tag = tag == 0x3FFFFFFFu ? 0u : tag;          // next tag - 1 = this tag
    w->t = w->t + 1;
  }
}

// ---------------------------------------------------------------------------
// route

// Message to node n for source s: bits 0..31 source, 32..39 mask of the
// node's destination partitions, 40..63 index (in s's destination list) of
// the node's first destination partition.
__device__ __forceinline__ uint32_t node_mask(const KParams& p, int64_t j, int64_t j1,
                                              uint32_t node) {
  uint32_t mask = 0;
  for (int64_t jj = j; jj < j1; ++jj) {
    const uint32_t vv = p.vp_part[jj];
    if (vv / p.G != node) break;
    mask |= 1u << (vv - p.G * node);
  }
  return mask;
}

__device__ __forceinline__ void bucket_put(const KParams& p, uint32_t node, uint32_t pos,
                                           uint64_t msg) {
  const uint64_t off = p.bucket_off[node];
  if (off + pos < p.bucket_off[node + 1]) p.bucket[off + pos] = msg;
  else atomicOr(&p.st->error, ERR_BUCKET);
}

// Two-level: block b takes a contiguous chunk of the fired sources and works
// in rounds of SB sources (a source emits at most n_nodes messages).  Within
// a round one wave per source finds the runs of equal node in its ascending
// destination list; the first lane of each run ORs the run into a mask and
// stages the message in LDS with its rank among the block's messages to that
// node.  One atomic per (round, node) then reserves the node's bucket space.
// Dynamic LDS: 2 * n_nodes counters + ROUTE_STAGE staged messages.
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_two_level(KParams p) {
  extern __shared__ uint64_t lds_u64[];
  uint64_t* s_msg = lds_u64;                                              // [ROUTE_STAGE]
  uint32_t* s_nr = reinterpret_cast<uint32_t*>(s_msg + ROUTE_STAGE);      // node | rank << 16
  uint32_t* l_cnt = s_nr + ROUTE_STAGE;                                   // [n_nodes]
  uint32_t* l_base = l_cnt + p.n_nodes;                                   // [n_nodes]
  __shared__ uint32_t l_total;
  constexpr uint32_t NW = ROUTE_THREADS / 64;
  const uint32_t nF = p.st->n_fired;
  const uint32_t row = p.st->cur_row;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t chunk = (nF + gridDim.x - 1) / gridDim.x;
  const uint32_t lo = min(blockIdx.x * chunk, nF), hi = min(lo + chunk, nF);
  const uint32_t SB = max(1u, ROUTE_STAGE / p.n_nodes);
  uint64_t l1 = 0, l2 = 0;
  for (uint32_t r0 = lo; r0 < hi; r0 += SB) {
    const uint32_t r1 = min(r0 + SB, hi);
    for (uint32_t i = tid; i < p.n_nodes; i += ROUTE_THREADS) l_cnt[i] = 0;
    if (tid == 0) l_total = 0;
    __syncthreads();
    for (uint32_t i = r0 + wave; i < r1; i += NW) {
      const uint32_t s = p.fired[i];
      const uint32_t own_node = static_cast<uint32_t>(p.part[s]) / p.G;
      const int64_t j0 = p.vp_ptr[s], j1 = p.vp_ptr[s + 1];
      for (int64_t jb = j0; jb < j1; jb += 64) {
        const int64_t j = jb + lane;
        if (j >= j1) continue;
        const uint32_t node = p.vp_part[j] / p.G;
        if (j != j0 && p.vp_part[j - 1] / p.G == node) continue;
        const uint64_t msg = (static_cast<uint64_t>(j - j0) << 40) |
                             (static_cast<uint64_t>(node_mask(p, j, j1, node)) << 32) | s;
        const uint32_t k = atomicAdd(&l_total, 1u);
        if (k < ROUTE_STAGE) {
          const uint32_t rk = atomicAdd(&l_cnt[node], 1u);
          s_msg[k] = msg;
          s_nr[k] = node | (rk << 16);
        } else {
          bucket_put(p, node, atomicAdd(p.bucket_cnt + node * CNT_STRIDE, 1u), msg);
        }
        if (node == own_node) ++l1; else ++l2;
      }
    }
    __syncthreads();
    for (uint32_t n = tid; n < p.n_nodes; n += ROUTE_THREADS) {
      const uint32_t c = l_cnt[n];
      if (c) l_base[n] = atomicAdd(p.bucket_cnt + n * CNT_STRIDE, c);
    }
    __syncthreads();
    const uint32_t staged = min(l_total, ROUTE_STAGE);
    for (uint32_t k = tid; k < staged; k += ROUTE_THREADS) {
      const uint32_t nr = s_nr[k];
      const uint32_t node = nr & 0xFFFFu;
      bucket_put(p, node, l_base[node] + (nr >> 16), s_msg[k]);
    }
    __syncthreads();
  }
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_MSG_L1, l1);
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_MSG_L2, l2);
}

// Two-level routing without LDS staging, for node counts whose counters do
// not fit LDS: one wave per source, one atomic per message.
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_two_level_direct(KParams p) {
  const uint32_t nF = p.st->n_fired;
  const uint32_t row = p.st->cur_row;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t n_waves = gridDim.x * (ROUTE_THREADS / 64);
  uint64_t l1 = 0, l2 = 0;
  for (uint32_t i = blockIdx.x * (ROUTE_THREADS / 64) + (threadIdx.x >> 6); i < nF; i += n_waves) {
    const uint32_t s = p.fired[i];
    const uint32_t own_node = static_cast<uint32_t>(p.part[s]) / p.G;
    const int64_t j0 = p.vp_ptr[s], j1 = p.vp_ptr[s + 1];
    for (int64_t jb = j0; jb < j1; jb += 64) {
      const int64_t j = jb + lane;
      if (j >= j1) continue;
      const uint32_t node = p.vp_part[j] / p.G;
      if (j != j0 && p.vp_part[j - 1] / p.G == node) continue;
      const uint64_t msg = (static_cast<uint64_t>(j - j0) << 40) |
                           (static_cast<uint64_t>(node_mask(p, j, j1, node)) << 32) | s;
      bucket_put(p, node, atomicAdd(p.bucket_cnt + node * CNT_STRIDE, 1u), msg);
      if (node == own_node) ++l1; else ++l2;
    }
  }
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_MSG_L1, l1);
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_MSG_L2, l2);
}

// Expansion at destination node n (grid x = chunks of the bucket, y = node):
// every set bit b of a message's mask appends (source, index of partition
// G*n + b in the source's destination list) to that partition's receive list.
// A block only touches the node's G partitions, so entries are staged in LDS
// and each round reserves with G atomics.
__global__ __launch_bounds__(ROUTE_THREADS) void k_expand(KParams p) {
  __shared__ uint64_t s_ent[ROUTE_STAGE];
  __shared__ uint16_t s_br[ROUTE_STAGE];       // b | rank << 3 (rank < ROUTE_STAGE)
  __shared__ uint32_t l_cnt[SNN_MAX_GPUS_PER_NODE], l_base[SNN_MAX_GPUS_PER_NODE];
  __shared__ uint32_t l_total;
  const uint32_t n = blockIdx.y;
  const uint32_t tid = threadIdx.x;
  const uint32_t row = p.st->cur_row;
  const uint64_t off = p.bucket_off[n];
  const uint64_t cap = p.bucket_off[n + 1] - off;
  const uint64_t cnt = min(static_cast<uint64_t>(p.bucket_cnt[n * CNT_STRIDE]), cap);
  const uint64_t per = (cnt + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = min(static_cast<uint64_t>(blockIdx.x) * per, cnt), hi = min(lo + per, cnt);
  const uint32_t MB = ROUTE_STAGE / p.G;      // a message yields at most G entries
  uint64_t entries = 0;
  for (uint64_t m0 = lo; m0 < hi; m0 += MB) {
    const uint64_t m1 = min(m0 + MB, hi);
    if (tid < SNN_MAX_GPUS_PER_NODE) l_cnt[tid] = 0;
    if (tid == 0) l_total = 0;
    __syncthreads();
    for (uint64_t m = m0 + tid; m < m1; m += ROUTE_THREADS) {
      const uint64_t msg = p.bucket[off + m];
      const uint64_t s = msg & 0xFFFFFFFFull;
      uint32_t mask = static_cast<uint32_t>(msg >> 32) & 0xFFu;
      uint64_t jrel = msg >> 40;
      while (mask) {
        const uint32_t b = __ffs(mask) - 1;
        mask &= mask - 1;
        if (b >= p.G || p.G * n + b >= p.P) {
          atomicOr(&p.st->error, ERR_ROUTE);
          continue;
        }
        const uint32_t k = atomicAdd(&l_total, 1u);
        const uint32_t rk = atomicAdd(&l_cnt[b], 1u);
        s_ent[k] = s | (jrel << 32);
        s_br[k] = static_cast<uint16_t>(b | (rk << 3));
        ++jrel;
        ++entries;
      }
    }
    __syncthreads();
    if (tid < p.G && l_cnt[tid])
      l_base[tid] = atomicAdd(p.recv_cnt + (p.G * n + tid) * CNT_STRIDE, l_cnt[tid]);
    __syncthreads();
    for (uint32_t k = tid; k < l_total; k += ROUTE_THREADS) {
      const uint32_t b = s_br[k] & 7u;
      const uint32_t part = p.G * n + b;
      const uint64_t pos = l_base[b] + (s_br[k] >> 3);
      const uint64_t roff = p.recv_off[part];
      if (roff + pos < p.recv_off[part + 1]) p.recv[roff + pos] = s_ent[k];
      else atomicOr(&p.st->error, ERR_RECV);
    }
    __syncthreads();
  }
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_RECV_ENTRIES, entries);
}

// Flat (direct peer-to-peer) routing: one wave per fired source, one receive
// entry (source, index in its destination list) per destination partition.
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_flat(KParams p) {
  const uint32_t nF = p.st->n_fired;
  const uint32_t row = p.st->cur_row;
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
        p.flat[off + pos] = static_cast<uint64_t>(s) | (static_cast<uint64_t>(j - j0) << 32);
      else
        atomicOr(&p.st->error, ERR_FLAT);
      ++flat;
    }
  }
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_FLAT_MSGS, flat);
}

// ---------------------------------------------------------------------------
// receive side: stage remote synapses per delay

// Block b of STAGE_BLOCKS owns a contiguous range of partitions and their
// receive lists.  For every entry (s, j): the receiving partition's synapses
// of source s are the row segment of s's j-th destination; each synapse is
// staged in LDS by delay and written to the block's own queue for that delay
// (no global atomics: the queue belongs to the block).  Rounds take one entry
// per thread; events beyond the LDS stage go straight to the queue.
__global__ __launch_bounds__(DELIVER_THREADS) void k_recv_stage(KParams p, int use_flat) {
  __shared__ Event s_ev[DELIVER_STAGE];
  __shared__ uint32_t s_dr[DELIVER_STAGE];     // (d - 1) | rank << 4
  __shared__ uint32_t s_pref[STAGE_PARTS + 1];
  __shared__ uint32_t l_cnt[SNN_MAX_DELAY], l_run[SNN_MAX_DELAY];
  __shared__ uint32_t l_total;
  const uint32_t tid = threadIdx.x, b = blockIdx.x;
  const uint32_t md = p.D - 1;
  const uint32_t slot0 = p.st->cur_slot;
  const uint32_t row = p.st->cur_row;
  const uint32_t ppb = (p.P + STAGE_BLOCKS - 1) / STAGE_BLOCKS;
  const uint32_t q0 = min(b * ppb, p.P), q1 = min(q0 + ppb, p.P);
  const uint64_t* lists = use_flat ? p.flat : p.recv;
  const uint32_t* cnts = use_flat ? p.flat_cnt : p.recv_cnt;
  if (tid == 0) {
    uint32_t acc = 0;
    for (uint32_t q = q0; q < q1; ++q) {
      s_pref[q - q0] = acc;
      const uint64_t cap = p.recv_off[q + 1] - p.recv_off[q];
      acc += static_cast<uint32_t>(min(static_cast<uint64_t>(cnts[q * CNT_STRIDE]), cap));
    }
    s_pref[q1 - q0] = acc;
  }
  if (tid < SNN_MAX_DELAY) l_run[tid] = 0;
  __syncthreads();
  const uint32_t n_ent = s_pref[q1 - q0];
  Event* queue = p.stage + static_cast<uint64_t>(b) * p.stage_cap;  // + (d-1)*STAGE_BLOCKS*cap
  const uint64_t qstride = static_cast<uint64_t>(STAGE_BLOCKS) * p.stage_cap;
  uint64_t events = 0;
  for (uint32_t e0 = 0; e0 < n_ent; e0 += DELIVER_THREADS) {
    if (tid < SNN_MAX_DELAY) l_cnt[tid] = 0;
    if (tid == 0) l_total = 0;
    __syncthreads();
    const uint32_t e = e0 + tid;
    if (e < n_ent) {
      uint32_t lo = 0, hi = q1 - q0;          // partition of entry e: s_pref[lo] <= e < s_pref[lo+1]
      while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (s_pref[mid] <= e) lo = mid; else hi = mid;
      }
      const uint32_t q = q0 + lo;
      const uint64_t ent = lists[p.recv_off[q] + (e - s_pref[lo])];
      const uint32_t s = static_cast<uint32_t>(ent);
      const int64_t jb = s < p.N ? p.vp_ptr[s] : 0, je = s < p.N ? p.vp_ptr[s + 1] : 0;
      const int64_t j = jb + static_cast<int64_t>(ent >> 32);
      if (s >= p.N || j >= je || p.vp_part[j] != q) {
        atomicOr(&p.st->error, ERR_ROUTE);
      } else {
        const uint64_t r0 = static_cast<uint64_t>(p.row_ptr[s]);
        const uint64_t a = r0 + p.vp_seg[j];
        const uint64_t z = j + 1 < je ? r0 + p.vp_seg[j + 1] : static_cast<uint64_t>(p.row_ptr[s + 1]);
        events += z - a;
        for (uint64_t x = a; x < z; ++x) {
          const uint32_t td = p.tgt_delay[x];
          const uint32_t d1 = (td >> 27) - 1;
          if (d1 >= md) {                      // delay outside [1, max_delay]
            atomicOr(&p.st->error, ERR_ROUTE);
            continue;
          }
          const Event ev{td & 0x07FFFFFFu, load_weight(p, x)};
          const uint32_t k = atomicAdd(&l_total, 1u);
          if (k < DELIVER_STAGE) {
            const uint32_t rk = atomicAdd(&l_cnt[d1], 1u);
            s_ev[k] = ev;
            s_dr[k] = d1 | (rk << 4);
          } else {
            uint32_t slot = slot0 + d1 + 1;
            if (slot >= p.D) slot -= p.D;
            ring_fallback(p, slot, ev.tgt, ev.w);
          }
        }
      }
    }
    __syncthreads();
    const uint32_t staged = min(l_total, DELIVER_STAGE);
    for (uint32_t k = tid; k < staged; k += DELIVER_THREADS) {
      const uint32_t d1 = s_dr[k] & 15u;
      const uint64_t pos = static_cast<uint64_t>(l_run[d1]) + (s_dr[k] >> 4);
      if (pos < p.stage_cap) {
        queue[d1 * qstride + pos] = s_ev[k];
      } else {
        uint32_t slot = slot0 + d1 + 1;
        if (slot >= p.D) slot -= p.D;
        ring_fallback(p, slot, s_ev[k].tgt, s_ev[k].w);
      }
    }
    __syncthreads();
    if (tid < md) l_run[tid] += l_cnt[tid];
    __syncthreads();
  }
  if (tid < md)
    p.stage_cnt[tid * STAGE_BLOCKS + b] =
        static_cast<uint32_t>(min(static_cast<uint64_t>(l_run[tid]), p.stage_cap));
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_REMOTE_EVENTS, events);
}

// ---------------------------------------------------------------------------
// deliver: per delay, counting-sort events by tile into private sub-bins

// Block (w, d): the delay-d run of the local segment of fired sources
// w, w + DELIVER_BLOCKS, ..., then the staging queues q = w (mod
// DELIVER_BLOCKS) of delay d.  Every event lands in ring slot (t + d) mod D,
// so the block counting-sorts them by tile in LDS and writes each tile's run
// into sub-bin (slot, tile, d, w).  That sub-bin is written by this block
// only, once per ring cycle, and read by the tile's update D - d steps later:
// positions and counts need no atomics.  Rounds are sized by a wave scan of
// the sources' run lengths so that they fit the LDS stage.
// Dynamic LDS: DELIVER_STAGE events + tile/rank words + 2 * n_tiles counters.
__global__ __launch_bounds__(DELIVER_THREADS) void k_deliver(KParams p) {
  extern __shared__ uint64_t lds_u64[];
  Event* s_ev = reinterpret_cast<Event*>(lds_u64);                        // [DELIVER_STAGE]
  uint32_t* s_tr = reinterpret_cast<uint32_t*>(s_ev + DELIVER_STAGE);     // tile | rank << 16
  uint32_t* l_cnt = s_tr + DELIVER_STAGE;                                 // [n_tiles]
  uint32_t* l_run = l_cnt + p.n_tiles;                                    // [n_tiles]
  __shared__ uint32_t l_total, s_m0, s_mn;
  constexpr uint32_t NW = DELIVER_THREADS / 64;
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t w = blockIdx.x, d = blockIdx.y + 1;

  const uint32_t nF = p.st->n_fired;
  uint32_t slot = p.st->cur_slot + d;
  if (slot >= p.D) slot -= p.D;
  const uint32_t row = p.st->cur_row;
  const uint32_t D = p.D;
  for (uint32_t i = tid; i < p.n_tiles; i += DELIVER_THREADS) l_run[i] = 0;
  uint64_t events = 0;

  // stage one event; events beyond the LDS stage go to the ring
  auto stage = [&](uint32_t tgt, float wt) {
    const uint32_t tile = tgt >> TILE_SHIFT;
    const uint32_t k = atomicAdd(&l_total, 1u);
    if (k < DELIVER_STAGE) {
      const uint32_t rk = atomicAdd(&l_cnt[tile], 1u);
      s_ev[k] = Event{tgt & (TILE - 1), wt};
      s_tr[k] = tile | (rk << 16);
    } else {
      ring_fallback(p, slot, tgt, wt);
    }
  };
  // write the staged round into the sub-bins and advance the running counts
  auto flush = [&]() {
    __syncthreads();
    const uint32_t staged = min(l_total, DELIVER_STAGE);
    for (uint32_t k = tid; k < staged; k += DELIVER_THREADS) {
      const uint32_t tile = s_tr[k] & 0xFFFFu;
      const uint64_t pos = static_cast<uint64_t>(l_run[tile]) + (s_tr[k] >> 16);
      if (pos < p.bin_cap) {
        p.bins[subbin(p, slot, tile, d, w) * p.bin_cap + pos] = s_ev[k];
      } else {
        ring_fallback(p, slot, (tile << TILE_SHIFT) | s_ev[k].tgt, s_ev[k].w);
      }
    }
    __syncthreads();
    for (uint32_t i = tid; i < p.n_tiles; i += DELIVER_THREADS) {
      l_run[i] += l_cnt[i];
      l_cnt[i] = 0;
    }
    if (tid == 0) l_total = 0;
    __syncthreads();
  };

  for (uint32_t i = tid; i < p.n_tiles; i += DELIVER_THREADS) l_cnt[i] = 0;
  if (tid == 0) l_total = 0;
  __syncthreads();

  // local synapses of the fired sources assigned to this block
  const uint32_t M = nF > w ? (nF - w + DELIVER_BLOCKS - 1) / DELIVER_BLOCKS : 0;
  uint32_t m_next = 0;
  while (m_next < M) {
    if (wave == 0) {
      const uint32_t m = m_next + lane;
      uint32_t len = 0;
      if (m < M) {
        const uint32_t s = p.fired[w + m * DELIVER_BLOCKS];
        len = p.delay_off[static_cast<uint64_t>(s) * D + d] -
              p.delay_off[static_cast<uint64_t>(s) * D + d - 1];
      }
      const uint32_t incl = wave_incl_scan(len);
      const uint32_t fit = __popcll(__ballot(m < M && incl <= DELIVER_STAGE));
      if (lane == 0) {
        s_m0 = m_next;
        s_mn = max(fit, 1u);
      }
    }
    __syncthreads();
    const uint32_t m0 = s_m0, mn = s_mn;
    for (uint32_t k = wave; k < mn; k += NW) {
      const uint32_t s = p.fired[w + (m0 + k) * DELIVER_BLOCKS];
      const uint64_t r0 = static_cast<uint64_t>(p.row_ptr[s]);
      const uint32_t a = p.delay_off[static_cast<uint64_t>(s) * D + d - 1];
      const uint32_t z = p.delay_off[static_cast<uint64_t>(s) * D + d];
      for (uint32_t x = a + lane; x < z; x += 64)
        stage(p.tgt_delay[r0 + x] & 0x07FFFFFFu, load_weight(p, r0 + x));
      if (lane == 0) events += z - a;
    }
    flush();
    m_next = m0 + mn;
  }

  // remote synapses staged by the receive side for this delay
  for (uint32_t q = w; q < STAGE_BLOCKS; q += DELIVER_BLOCKS) {
    const uint32_t c = p.stage_cnt[(d - 1) * STAGE_BLOCKS + q];
    const Event* src = p.stage + (static_cast<uint64_t>(d - 1) * STAGE_BLOCKS + q) * p.stage_cap;
    for (uint32_t e0 = 0; e0 < c; e0 += DELIVER_STAGE) {
      const uint32_t e1 = min(e0 + DELIVER_STAGE, c);
      for (uint32_t e = e0 + tid; e < e1; e += DELIVER_THREADS) stage(src[e].tgt, src[e].w);
      flush();
    }
  }

  // publish this block's counts for slot `slot`, every tile (zeros included)
  for (uint32_t i = tid; i < p.n_tiles; i += DELIVER_THREADS)
    p.bin_cnt[subbin(p, slot, i, d, w)] =
        static_cast<uint32_t>(min(static_cast<uint64_t>(l_run[i]), p.bin_cap));
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_LOCAL_EVENTS, events);
}

// Moves every pending binned event into the dense ring (for read-back) and
// empties those bins.  Grid: x = tile, y = slot.  Bins are not cleared when
// consumed, so only some are pending: slot s is consumed k steps from now
// (k = (s - next slot) mod D), and its bin of delay d has been written for
// that step only if d > k (it is written at step s - d); the others still
// hold input already consumed.
__global__ __launch_bounds__(256) void k_flush(KParams p) {
  const uint32_t tile = blockIdx.x, slot = blockIdx.y;
  const uint32_t next = p.st->slot;
  const uint32_t ahead = slot >= next ? slot - next : slot + p.D - next;
  const uint32_t md = p.D - 1;
  __shared__ uint32_t any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (uint32_t d = ahead + 1; d <= md; ++d) {
    for (uint32_t w = 0; w < DELIVER_BLOCKS; ++w) {
      const uint64_t sb = subbin(p, slot, tile, d, w);
      const uint32_t c = min(p.bin_cnt[sb], static_cast<uint32_t>(p.bin_cap));
      const Event* ev = p.bins + sb * p.bin_cap;
      for (uint32_t e = threadIdx.x; e < c; e += 256)
        unsafeAtomicAdd(p.ring + slot * p.ring_stride + (tile << TILE_SHIFT) + ev[e].tgt,
                        ev[e].w);
      if (c && threadIdx.x == 0) any = 1;
      __syncthreads();
      if (threadIdx.x == 0) p.bin_cnt[sb] = 0;
    }
  }
  if (threadIdx.x == 0 && any) p.dirty[slot * p.n_tiles + tile] = 1u;
}

// ---------------------------------------------------------------------------
// launchers

uint32_t tiles_of(uint32_t n) { return (n + TILE - 1) / TILE; }

hipError_t launch_update(const KParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(p.n_tiles), dim3(UPDATE_THREADS), 0, s, p);
  return hipGetLastError();
}

size_t route_lds_bytes(const KParams& p) {
  return ROUTE_STAGE * (sizeof(uint64_t) + sizeof(uint32_t)) + 2ull * p.n_nodes * sizeof(uint32_t);
}

hipError_t launch_route(const KParams& p, int mode, hipStream_t s) {
  if (mode == SNN_ROUTE_TWO_LEVEL || mode == SNN_ROUTE_BOTH) {
    if (p.n_nodes <= ROUTE_MAX_NODES_LDS)
      hipLaunchKernelGGL(k_route_two_level, dim3(ROUTE_BLOCKS), dim3(ROUTE_THREADS),
                         route_lds_bytes(p), s, p);
    else
      hipLaunchKernelGGL(k_route_two_level_direct, dim3(1024), dim3(ROUTE_THREADS), 0, s, p);
    hipLaunchKernelGGL(k_expand, dim3(EXPAND_BLOCKS, p.n_nodes), dim3(ROUTE_THREADS), 0, s, p);
  }
  if (mode == SNN_ROUTE_FLAT || mode == SNN_ROUTE_BOTH)
    hipLaunchKernelGGL(k_route_flat, dim3(1024), dim3(ROUTE_THREADS), 0, s, p);
  return hipGetLastError();
}

size_t deliver_lds_bytes(const KParams& p) {
  return DELIVER_STAGE * (sizeof(Event) + sizeof(uint32_t)) + 2ull * p.n_tiles * sizeof(uint32_t);
}

hipError_t launch_deliver(const KParams& p, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_recv_stage, dim3(STAGE_BLOCKS), dim3(DELIVER_THREADS), 0, s, p,
                     mode == SNN_ROUTE_FLAT ? 1 : 0);
  hipLaunchKernelGGL(k_deliver, dim3(DELIVER_BLOCKS, p.D - 1), dim3(DELIVER_THREADS),
                     deliver_lds_bytes(p), s, p);
  return hipGetLastError();
}

hipError_t prepare_kernels(const KParams& p) {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_route_two_level),
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     static_cast<int>(route_lds_bytes(p)));
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void*>(&k_deliver),
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             static_cast<int>(deliver_lds_bytes(p)));
}

hipError_t launch_flush(const KParams& p, hipStream_t s) {
  hipLaunchKernelGGL(k_flush, dim3(p.n_tiles, p.D), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace snn
