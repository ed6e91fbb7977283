// snn_kernels.hip — the per-step kernels for gfx950 (wave64, CDNA4).
//
//   update   LIF update + threshold of every neuron, fused with the ascending
//            compaction of fired ids (wave ballots, block scan, decoupled
//            look-back across blocks)
//   route    two-level: one (source, node mask) message per destination node
//            into per-node buckets (Sec. IV-B), then mask expansion into
//            per-partition receive lists (the bridge's forwarding);
//            flat: one receive entry per destination partition
//   deliver  own-partition synapses of every fired source, then the
//            synapses reached through the receive lists, atomically added
//            into the delay ring
//
// The work is sparse gather/scatter bound by HBM and L2 atomics; there is no
// dense contraction, so no MFMA.  Compiled with -ffp-contract=off: the
// membrane update rounds after every operation, exactly as specified.
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

__device__ __forceinline__ float load_weight(const KParams& p, uint64_t e) {
  if (p.bf16) {
    const uint16_t b = static_cast<const uint16_t*>(p.weight)[e];
    return __uint_as_float(static_cast<uint32_t>(b) << 16);
  }
  return static_cast<const float*>(p.weight)[e];
}

__device__ __forceinline__ void ring_add(const KParams& p, uint32_t slot0, uint32_t td,
                                         float w) {
  const uint32_t tgt = td & 0x07FFFFFFu;
  uint32_t slot = slot0 + (td >> 27);
  if (slot >= p.D) slot -= p.D;
  unsafeAtomicAdd(p.ring + slot * p.ring_stride + tgt, w);
}

// Adds a per-thread counter into a global u64 with one atomic per wave.
__device__ __forceinline__ void add_stat(uint64_t* dst, uint64_t v) {
  v = wave_sum64(v);
  if ((threadIdx.x & 63) == 0 && v) atomicAdd(reinterpret_cast<unsigned long long*>(dst), v);
}

// ---------------------------------------------------------------------------
// update: neuron update, threshold, ascending compaction of fired ids

// Look-back word: [63:34] step tag, [33:32] status, [31:0] count.
constexpr uint32_t LB_AGG = 1u, LB_INCL = 2u;

__device__ __forceinline__ uint64_t lb_pack(uint32_t tag, uint32_t status, uint32_t v) {
  return (static_cast<uint64_t>(tag) << 34) | (static_cast<uint64_t>(status) << 32) | v;
}

// Wave 0 of block b: publishes the block's count, walks back over the
// predecessors 64 at a time until an inclusive prefix closes the window, and
// publishes the inclusive prefix.  Returns the exclusive prefix.
__device__ uint32_t lookback_exclusive(uint64_t* lb, uint32_t b, uint32_t agg, uint32_t tag) {
  const int lane = threadIdx.x & 63;
  if (b == 0) {
    if (lane == 0)
      __hip_atomic_store(lb, lb_pack(tag, LB_INCL, agg), __ATOMIC_RELEASE,
                         __HIP_MEMORY_SCOPE_AGENT);
    return 0;
  }
  if (lane == 0)
    __hip_atomic_store(lb + b, lb_pack(tag, LB_AGG, agg), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  uint32_t excl = 0;
  int64_t j = static_cast<int64_t>(b) - 1;
  while (true) {
    const int64_t idx = j - lane;
    uint64_t w = idx >= 0 ? __hip_atomic_load(lb + idx, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)
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
    __hip_atomic_store(lb + b, lb_pack(tag, LB_INCL, excl + agg), __ATOMIC_RELEASE,
                       __HIP_MEMORY_SCOPE_AGENT);
  return excl;
}

// One thread owns NPT neurons as NPT/4 quads.  Quad q of thread tid covers
// neurons blk0 + q*4*UPDATE_THREADS + 4*tid .. +3, so every load and store
// instruction of a wave touches one contiguous 1 KiB span.  Ids are ordered
// quad-major across the block, which the compaction follows.
template <int NPT>
__global__ __launch_bounds__(UPDATE_THREADS) void k_update(KParams p) {
  static_assert(NPT % 4 == 0 && NPT >= 4, "NPT is a multiple of 4");
  constexpr int NQ = NPT / 4;
  constexpr int NW = UPDATE_THREADS / 64;
  __shared__ uint32_t s_cnt[NQ][NW];
  __shared__ uint32_t s_excl;

  // Read once: the last block advances both when the step is complete.
  const uint64_t t = __hip_atomic_load(&p.st->t, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint64_t log_base =
      __hip_atomic_load(&p.st->log_total, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  const uint32_t slot = static_cast<uint32_t>(t % p.D);
  const uint32_t row = static_cast<uint32_t>(t % p.log_steps);
  const uint32_t tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const uint32_t blk0 = blockIdx.x * (UPDATE_THREADS * NPT);

  // Per-step counters of the routing and delivery kernels that follow.
  if (blockIdx.x == 0) {
    for (uint32_t i = tid; i < p.n_nodes; i += UPDATE_THREADS) p.bucket_cnt[i] = 0;
    for (uint32_t i = tid; i < p.P; i += UPDATE_THREADS) {
      p.recv_cnt[i] = 0;
      p.flat_cnt[i] = 0;
    }
    if (tid >= 1 && tid < SNN_NSTAT) p.stats[static_cast<uint64_t>(row) * SNN_NSTAT + tid] = 0;
  }

  uint32_t thr_raster = 0;
  if (p.forced) thr_raster = (t % p.raster_period) < p.raster_on ? p.raster_on_thr : p.raster_off_thr;
  float* ring_slot = p.ring + static_cast<uint64_t>(slot) * p.ring_stride;

  uint32_t fire_bits = 0;   // bit 4q + k: neuron k of quad q fired
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const uint32_t i0 = blk0 + q * (4 * UPDATE_THREADS) + 4 * tid;
    // Philox counter word 0 is i0 / 4: one call serves the quad's 4 neurons.
    const uint4 rnd = philox4x32_10(i0 >> 2, static_cast<uint32_t>(t), STREAM_POISSON, 0u,
                                    p.seed_lo, p.seed_hi);
    uint4 rnd2 = make_uint4(0, 0, 0, 0);
    if (p.forced)
      rnd2 = philox4x32_10(i0 >> 2, static_cast<uint32_t>(t), STREAM_RASTER, 0u, p.seed_lo,
                           p.seed_hi);
    const uint32_t r1[4] = {rnd.x, rnd.y, rnd.z, rnd.w};
    const uint32_t r2[4] = {rnd2.x, rnd2.y, rnd2.z, rnd2.w};
    float uu[4] = {0.f, 0.f, 0.f, 0.f}, syn[4] = {0.f, 0.f, 0.f, 0.f};
    uint32_t rf[4] = {0, 0, 0, 0};
    const bool full = i0 + 4 <= p.N;
    if (full) {
      const float4 u4 = *reinterpret_cast<const float4*>(p.u + i0);
      const float4 s4 = *reinterpret_cast<const float4*>(ring_slot + i0);
      const uint32_t r4 = *reinterpret_cast<const uint32_t*>(p.ref + i0);
      uu[0] = u4.x; uu[1] = u4.y; uu[2] = u4.z; uu[3] = u4.w;
      syn[0] = s4.x; syn[1] = s4.y; syn[2] = s4.z; syn[3] = s4.w;
#pragma unroll
      for (int k = 0; k < 4; ++k) rf[k] = (r4 >> (8 * k)) & 0xFFu;
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i0 + k < p.N) {
          uu[k] = p.u[i0 + k];
          syn[k] = ring_slot[i0 + k];
          rf[k] = p.ref[i0 + k];
        }
    }
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
      *reinterpret_cast<float4*>(ring_slot + i0) = make_float4(0.f, 0.f, 0.f, 0.f);
      *reinterpret_cast<uint32_t*>(p.ref + i0) =
          rf[0] | (rf[1] << 8) | (rf[2] << 16) | (rf[3] << 24);
    } else {
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (i0 + k < p.N) {
          p.u[i0 + k] = uu[k];
          ring_slot[i0 + k] = 0.f;
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
  const uint32_t tag = static_cast<uint32_t>(t % 0x3FFFFFFFull) + 1u;
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
          if (p.log_cap) p.log[(log_base + pos) % p.log_cap] = i0 + k;
          ++pos;
        }
    }
  }

  // The last block holds the step total once its look-back is done; every
  // other block has read t and log_total by then (they published first).
  if (blockIdx.x == gridDim.x - 1 && tid == 0) {
    const uint32_t n = s_excl + block_tot;
    p.st->n_fired = n;
    p.stats[static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_SPIKES] = n;
    p.log_off[row] = log_base;
    if (p.log_cap && n > p.log_cap) atomicOr(&p.st->error, ERR_LOG);
    p.st->log_total = log_base + n;
    p.st->t = t + 1;
  }
}

// ---------------------------------------------------------------------------
// route

// Two-level: one wave per fired source.  The source's destination
// partitions are ascending, so the partitions of one node are a contiguous
// run; the first lane of each run ORs the run into a mask and emits one
// message to that node's bucket.
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_two_level(KParams p) {
  const uint32_t nF = p.st->n_fired;
  const uint32_t row = static_cast<uint32_t>((p.st->t - 1) % p.log_steps);
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
      const uint32_t v = p.vp_part[j];
      const uint32_t node = v / p.G;
      if (j != j0 && p.vp_part[j - 1] / p.G == node) continue;
      uint32_t mask = 0;
      for (int64_t jj = j; jj < j1; ++jj) {
        const uint32_t vv = p.vp_part[jj];
        if (vv / p.G != node) break;
        mask |= 1u << (vv - p.G * node);
      }
      const uint32_t pos = atomicAdd(p.bucket_cnt + node, 1u);
      const uint64_t off = p.bucket_off[node];
      if (off + pos < p.bucket_off[node + 1])
        p.bucket[off + pos] = (static_cast<uint64_t>(j - j0) << 40) |
                              (static_cast<uint64_t>(mask) << 32) | s;
      else
        atomicOr(&p.st->error, ERR_BUCKET);
      if (node == own_node) ++l1; else ++l2;
    }
  }
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_MSG_L1, l1);
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_MSG_L2, l2);
}

// Expansion at each destination node: every set bit b of a message's mask
// appends the source to the receive list of partition G*n + b.
// Grid: x = chunks of a bucket, y = node.
__global__ __launch_bounds__(ROUTE_THREADS) void k_expand(KParams p) {
  const uint32_t n = blockIdx.y;
  const uint32_t row = static_cast<uint32_t>((p.st->t - 1) % p.log_steps);
  const uint64_t off = p.bucket_off[n];
  const uint64_t cap = p.bucket_off[n + 1] - off;
  const uint64_t cnt = min(static_cast<uint64_t>(p.bucket_cnt[n]), cap);
  uint64_t entries = 0;
  for (uint64_t m = static_cast<uint64_t>(blockIdx.x) * ROUTE_THREADS + threadIdx.x; m < cnt;
       m += static_cast<uint64_t>(gridDim.x) * ROUTE_THREADS) {
    const uint64_t msg = p.bucket[off + m];
    const uint32_t s = static_cast<uint32_t>(msg);
    uint32_t mask = static_cast<uint32_t>(msg >> 32) & 0xFFu;
    while (mask) {
      const uint32_t b = __ffs(mask) - 1;
      mask &= mask - 1;
      const uint32_t part = p.G * n + b;
      if (b >= p.G || part >= p.P) {
        atomicOr(&p.st->error, ERR_ROUTE);
        continue;
      }
      const uint32_t pos = atomicAdd(p.recv_cnt + part, 1u);
      const uint64_t roff = p.recv_off[part];
      if (roff + pos < p.recv_off[part + 1]) p.recv[roff + pos] = s;
      else atomicOr(&p.st->error, ERR_RECV);
      ++entries;
    }
  }
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_RECV_ENTRIES, entries);
}

// Flat: one wave per fired source, one receive entry per destination partition.
__global__ __launch_bounds__(ROUTE_THREADS) void k_route_flat(KParams p) {
  const uint32_t nF = p.st->n_fired;
  const uint32_t row = static_cast<uint32_t>((p.st->t - 1) % p.log_steps);
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t n_waves = gridDim.x * (ROUTE_THREADS / 64);
  uint64_t flat = 0;
  for (uint32_t i = blockIdx.x * (ROUTE_THREADS / 64) + (threadIdx.x >> 6); i < nF; i += n_waves) {
    const uint32_t s = p.fired[i];
    const int64_t j0 = p.vp_ptr[s], j1 = p.vp_ptr[s + 1];
    for (int64_t j = j0 + lane; j < j1; j += 64) {
      const uint32_t v = p.vp_part[j];
      const uint32_t pos = atomicAdd(p.flat_cnt + v, 1u);
      const uint64_t off = p.recv_off[v];
      if (off + pos < p.recv_off[v + 1]) p.flat[off + pos] = s;
      else atomicOr(&p.st->error, ERR_FLAT);
      ++flat;
    }
  }
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_FLAT_MSGS, flat);
}

// ---------------------------------------------------------------------------
// deliver

// Own-partition synapses: one block per fired source (grid-stride), threads
// sweep the contiguous local segment of its row.
__global__ __launch_bounds__(DELIVER_THREADS) void k_deliver_local(KParams p) {
  const uint32_t nF = p.st->n_fired;
  const uint64_t tc = p.st->t - 1;
  const uint32_t slot0 = static_cast<uint32_t>(tc % p.D);
  const uint32_t row = static_cast<uint32_t>(tc % p.log_steps);
  uint64_t events = 0;
  for (uint32_t i = blockIdx.x; i < nF; i += gridDim.x) {
    const uint32_t s = p.fired[i];
    const uint64_t r0 = static_cast<uint64_t>(p.row_ptr[s]);
    const uint32_t nl = p.n_local[s];
    for (uint32_t e = threadIdx.x; e < nl; e += DELIVER_THREADS)
      ring_add(p, slot0, p.tgt_delay[r0 + e], load_weight(p, r0 + e));
    if (threadIdx.x == 0) events += nl;
  }
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_LOCAL_EVENTS, events);
}

// Receive side: for every entry s in partition q's list, find q in s's
// destination list (binary search; the receiving GPU's lookup of its incoming
// synapses of s) and sweep that row segment.  Grid: x = chunks, y = partition.
__global__ __launch_bounds__(DELIVER_THREADS) void k_deliver_recv(KParams p, int use_flat) {
  const uint32_t q = blockIdx.y;
  const uint64_t tc = p.st->t - 1;
  const uint32_t slot0 = static_cast<uint32_t>(tc % p.D);
  const uint32_t row = static_cast<uint32_t>(tc % p.log_steps);
  const uint32_t* list = use_flat ? p.flat : p.recv;
  const uint32_t* cntp = use_flat ? p.flat_cnt : p.recv_cnt;
  const uint64_t off = p.recv_off[q];
  const uint64_t cnt = min(static_cast<uint64_t>(cntp[q]), p.recv_off[q + 1] - off);
  uint64_t events = 0;
  for (uint64_t m = static_cast<uint64_t>(blockIdx.x) * DELIVER_THREADS + threadIdx.x; m < cnt;
       m += static_cast<uint64_t>(gridDim.x) * DELIVER_THREADS) {
    const uint32_t s = list[off + m];
    int64_t lo = p.vp_ptr[s], hi = p.vp_ptr[s + 1];   // search [lo, hi)
    const int64_t j1 = hi;
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if (p.vp_part[mid] < q) lo = mid + 1; else hi = mid;
    }
    if (lo >= j1 || p.vp_part[lo] != q) {
      atomicOr(&p.st->error, ERR_ROUTE);
      continue;
    }
    const uint64_t r0 = static_cast<uint64_t>(p.row_ptr[s]);
    const uint64_t e0 = r0 + p.vp_seg[lo];
    const uint64_t e1 = lo + 1 < j1 ? r0 + p.vp_seg[lo + 1] : static_cast<uint64_t>(p.row_ptr[s + 1]);
    for (uint64_t e = e0; e < e1; ++e) ring_add(p, slot0, p.tgt_delay[e], load_weight(p, e));
    events += e1 - e0;
  }
  add_stat(p.stats + static_cast<uint64_t>(row) * SNN_NSTAT + SNN_STAT_REMOTE_EVENTS, events);
}

// ---------------------------------------------------------------------------
// launchers

uint32_t update_blocks(uint32_t n, int npt) {
  const uint32_t per = UPDATE_THREADS * static_cast<uint32_t>(npt);
  return (n + per - 1) / per;
}

hipError_t launch_update(const KParams& p, int npt, hipStream_t s) {
  const dim3 grid(update_blocks(p.N, npt)), block(UPDATE_THREADS);
  switch (npt) {
    case 4: hipLaunchKernelGGL(k_update<4>, grid, block, 0, s, p); break;
    case 8: hipLaunchKernelGGL(k_update<8>, grid, block, 0, s, p); break;
    case 16: hipLaunchKernelGGL(k_update<16>, grid, block, 0, s, p); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_route(const KParams& p, int mode, hipStream_t s) {
  const uint32_t route_blocks = 1024;
  if (mode == SNN_ROUTE_TWO_LEVEL || mode == SNN_ROUTE_BOTH) {
    hipLaunchKernelGGL(k_route_two_level, dim3(route_blocks), dim3(ROUTE_THREADS), 0, s, p);
    hipLaunchKernelGGL(k_expand, dim3(8, p.n_nodes), dim3(ROUTE_THREADS), 0, s, p);
  }
  if (mode == SNN_ROUTE_FLAT || mode == SNN_ROUTE_BOTH)
    hipLaunchKernelGGL(k_route_flat, dim3(route_blocks), dim3(ROUTE_THREADS), 0, s, p);
  return hipGetLastError();
}

hipError_t launch_deliver(const KParams& p, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_deliver_local, dim3(2048), dim3(DELIVER_THREADS), 0, s, p);
  hipLaunchKernelGGL(k_deliver_recv, dim3(4, p.P), dim3(DELIVER_THREADS), 0, s, p,
                     mode == SNN_ROUTE_FLAT ? 1 : 0);
  return hipGetLastError();
}

}  // namespace snn
