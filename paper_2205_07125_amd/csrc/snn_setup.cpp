// snn_setup.cpp — host setup of the network arrays (include/snn_setup.h).
// Regenerates the seeded synapse list twice: pass 1 counts out-degrees, pass
// 2 places each synapse in its source row; rows are then sorted into
// [own partition | destination partitions ascending] and the destination
// lists and exact per-step capacity bounds are derived.
#include <omp.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

#include "snn_setup.h"

extern "C" {
#include "synth.h"
}

extern "C" snn_status snn_fail_v(snn_status s, const char* fmt, va_list ap);

namespace {

snn_status fail(snn_status s, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  snn_fail_v(s, fmt, ap);
  va_end(ap);
  return s;
}

// Round-to-nearest-even of a binary32 value to bfloat16 bits (the upper half
// of the binary32 encoding); NaN stays a quiet NaN.
uint16_t to_bf16(float x) {
  uint32_t b;
  std::memcpy(&b, &x, 4);
  if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu)) return uint16_t((b >> 16) | 0x40u);
  const uint32_t lsb = (b >> 16) & 1u;
  b += 0x7FFFu + lsb;
  return uint16_t(b >> 16);
}

// Progress lines for passes that take minutes at 5e9-1e10 synapses.
struct Progress {
  const char* what;
  int64_t total;
  bool on;
  int64_t done = 0;
  int next = 1;
  Progress(const char* w, int64_t t, bool v) : what(w), total(t), on(v) {}
  void add(int64_t n) {
    if (!on) return;
    const int64_t d = __atomic_add_fetch(&done, n, __ATOMIC_RELAXED);
    const int tenth = int(10 * d / (total ? total : 1));
    int cur = __atomic_load_n(&next, __ATOMIC_RELAXED);
    while (tenth >= cur && cur <= 10) {
      if (__atomic_compare_exchange_n(&next, &cur, cur + 1, false, __ATOMIC_RELAXED,
                                      __ATOMIC_RELAXED)) {
        std::fprintf(stderr, "[setup] %s %d%%\n", what, 10 * cur);
        std::fflush(stderr);
        cur += 1;
      }
    }
  }
};

struct RowItem {
  uint64_t key;   // (partition tag << 32) | tgt_delay; tag 0 = own partition
  uint32_t w;     // weight bits
  bool operator<(const RowItem& o) const { return key != o.key ? key < o.key : w < o.w; }
};

}  // namespace

struct snn_setup {
  snn_setup_spec spec;
  syn_gen* gen = nullptr;
  uint32_t N = 0, P = 0, G = 0, n_nodes = 0;
  int threads = 1;
  std::vector<int64_t> row_ptr;     // N+1
  std::vector<uint16_t> tag;        // nnz, after fill_rows: 0 own, else partition + 1
  std::vector<uint32_t> n_vp;       // N, distinct destination partitions per source
  std::vector<uint64_t> bucket_cap; // n_nodes
  std::vector<uint64_t> recv_cap;   // P
  uint64_t nnz = 0, pairs = 0, bucket_total = 0, recv_total = 0;
  double input_bound = 0.0;         // max over targets of the sum of |w| of their inputs
  bool rows_done = false;
};

extern "C" {

snn_status snn_setup_create(const snn_setup_spec* spec, const uint32_t* part_start,
                            const double* cross_frac, const int32_t* part_map,
                            snn_setup_handle* out) {
  if (!spec || !out) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (spec->n_neurons < 2 || spec->n_neurons > SNN_MAX_NEURONS)
    return fail(SNN_ERR_INVALID_ARG, "n_neurons=%u outside [2, 2^27]", spec->n_neurons);
  if (spec->max_delay == 0 || spec->max_delay > SNN_MAX_DELAY)
    return fail(SNN_ERR_INVALID_ARG, "max_delay=%u outside [1, 15]", spec->max_delay);
  if (spec->gpus_per_node == 0 || spec->gpus_per_node > SNN_MAX_GPUS_PER_NODE)
    return fail(SNN_ERR_INVALID_ARG, "gpus_per_node=%u outside [1, %u]", spec->gpus_per_node,
                SNN_MAX_GPUS_PER_NODE);
  if (spec->n_partitions == 0 || spec->n_partitions > SNN_MAX_PARTITIONS)
    return fail(SNN_ERR_INVALID_ARG, "n_partitions=%u outside [1, 65535]", spec->n_partitions);
  if (spec->weight_type != SNN_W_FP32 && spec->weight_type != SNN_W_BF16)
    return fail(SNN_ERR_INVALID_ARG, "weight_type=%u", spec->weight_type);
  syn_spec gs;
  gs.seed = spec->seed;
  gs.n_neurons = spec->n_neurons;
  gs.k_in = spec->k_in;
  gs.max_delay = spec->max_delay;
  gs.n_partitions = spec->n_partitions;
  gs.topology = spec->topology;
  gs.vp_set_size = spec->vp_set_size;
  gs.remote_frac = spec->remote_frac;
  gs.w_exc = spec->w_exc;
  gs.w_inh = spec->w_inh;
  gs.w_jitter = spec->w_jitter;
  gs.n_clusters = spec->n_clusters;
  gs.p_in = spec->p_in;
  syn_gen* gen = syn_create(&gs, part_start, cross_frac);
  if (!gen) return fail(SNN_ERR_INVALID_ARG, "network description rejected by the generator");
  if (part_map && syn_set_part_map(gen, part_map) != 0) {
    syn_destroy(gen);
    return fail(SNN_ERR_INVALID_ARG, "partition map rejected (entries in [0, n_partitions), "
                "materialised or clustered topology only)");
  }

  snn_setup* h = new (std::nothrow) snn_setup();
  if (!h) {
    syn_destroy(gen);
    return fail(SNN_ERR_INVALID_ARG, "out of host memory");
  }
  h->spec = *spec;
  h->gen = gen;
  h->N = spec->n_neurons;
  h->P = spec->n_partitions;
  h->G = spec->gpus_per_node;
  h->n_nodes = (h->P + h->G - 1) / h->G;
  h->threads = spec->n_threads ? int(spec->n_threads) : omp_get_max_threads();
  const uint32_t N = h->N, K = spec->k_in;

  // Pass 1: out-degree of every source.
  std::vector<uint32_t> outdeg(N, 0);
  uint32_t* od = outdeg.data();
  Progress prog("count", N, spec->verbose != 0);
#pragma omp parallel for num_threads(h->threads) schedule(dynamic, 256)
  for (int64_t t = 0; t < int64_t(N); ++t) {
    for (uint32_t k = 0; k < K; ++k) {
      uint32_t src, d, vp;
      float w;
      syn_edge(gen, uint32_t(t), k, &src, &d, &vp, &w);
      __atomic_fetch_add(od + src, 1u, __ATOMIC_RELAXED);
    }
    if ((t & 4095) == 0) prog.add(std::min<int64_t>(4096, int64_t(N) - t));
  }
  h->row_ptr.assign(size_t(N) + 1, 0);
  for (uint32_t i = 0; i < N; ++i) h->row_ptr[i + 1] = h->row_ptr[i] + od[i];
  h->nnz = uint64_t(h->row_ptr[N]);
  *out = h;
  return SNN_OK;
}

snn_status snn_setup_sizes(snn_setup_handle h, uint64_t* nnz, uint64_t* pairs,
                           uint64_t* bucket_total, uint64_t* recv_total) {
  if (!h) return fail(SNN_ERR_INVALID_ARG, "handle is NULL");
  if (nnz) *nnz = h->nnz;
  if (pairs) *pairs = h->pairs;
  if (bucket_total) *bucket_total = h->bucket_total;
  if (recv_total) *recv_total = h->recv_total;
  return SNN_OK;
}

snn_status snn_setup_input_bound(snn_setup_handle h, float* bound) {
  if (!h || !bound) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  if (!h->rows_done) return fail(SNN_ERR_BAD_STATE, "input bound needs snn_setup_fill_rows first");
  float b = float(h->input_bound);
  if (double(b) < h->input_bound) b = std::nextafter(b, INFINITY);
  *bound = b;
  return SNN_OK;
}

snn_status snn_setup_fill_rows(snn_setup_handle h, int64_t* row_ptr, uint32_t* n_local,
                               uint16_t* delay_off, uint32_t* tgt_delay, void* weight) {
  if (!h || !row_ptr || !n_local || !delay_off || !tgt_delay || !weight)
    return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  const uint32_t N = h->N, K = h->spec.k_in, P = h->P, G = h->G, n_nodes = h->n_nodes;
  const uint32_t md = h->spec.max_delay;
  int too_long = 0;
  const bool bf16 = h->spec.weight_type == SNN_W_BF16;
  try {
    h->tag.assign(h->nnz, 0);
    h->n_vp.assign(N, 0);
  } catch (const std::bad_alloc&) {
    return fail(SNN_ERR_INVALID_ARG, "out of host memory for %llu synapse tags",
                (unsigned long long)h->nnz);
  }
  std::memcpy(row_ptr, h->row_ptr.data(), sizeof(int64_t) * (size_t(N) + 1));
  std::vector<uint64_t> cursor(h->row_ptr.begin(), h->row_ptr.end() - 1);
  uint64_t* cur = cursor.data();
  uint16_t* tag = h->tag.data();
  float* wf = static_cast<float*>(weight);
  uint16_t* wb = static_cast<uint16_t*>(weight);
  syn_gen* gen = h->gen;

  // Pass 2: place every synapse in its source row (order fixed by the sort),
  // and bound each target's input in one step by the sum of its |w|.
  Progress prog("place", N, h->spec.verbose != 0);
  double bound = 0.0;
#pragma omp parallel for num_threads(h->threads) schedule(dynamic, 256) reduction(max : bound)
  for (int64_t t = 0; t < int64_t(N); ++t) {
    if ((t & 4095) == 0) prog.add(std::min<int64_t>(4096, int64_t(N) - t));
    double in_abs = 0.0;
    for (uint32_t k = 0; k < K; ++k) {
      uint32_t src, d, vp;
      float w;
      syn_edge(gen, uint32_t(t), k, &src, &d, &vp, &w);
      const uint64_t at = __atomic_fetch_add(cur + src, 1ull, __ATOMIC_RELAXED);
      tgt_delay[at] = (d << 27) | uint32_t(t);
      tag[at] = vp == syn_part_of(gen, src) ? 0 : uint16_t(vp + 1);
      if (bf16) {
        const uint16_t b = to_bf16(w);
        wb[at] = b;
        uint32_t bits = uint32_t(b) << 16;
        float wr;
        std::memcpy(&wr, &bits, 4);
        in_abs += std::fabs(double(wr));
      } else {
        wf[at] = w;
        in_abs += std::fabs(double(w));
      }
    }
    bound = std::max(bound, in_abs);
  }
  h->input_bound = bound;

  // Sort rows; count own-partition synapses, destination partitions, and the
  // per-node / per-partition capacity bounds.
  std::vector<std::vector<uint64_t>> bcap(h->threads, std::vector<uint64_t>(n_nodes, 0));
  std::vector<std::vector<uint64_t>> rcap(h->threads, std::vector<uint64_t>(P, 0));
  Progress sprog("sort", N, h->spec.verbose != 0);
#pragma omp parallel num_threads(h->threads)
  {
    std::vector<RowItem> items;
    std::vector<uint64_t>& bc = bcap[omp_get_thread_num()];
    std::vector<uint64_t>& rc = rcap[omp_get_thread_num()];
#pragma omp for schedule(dynamic, 256)
    for (int64_t s = 0; s < int64_t(N); ++s) {
      if ((s & 4095) == 0) sprog.add(std::min<int64_t>(4096, int64_t(N) - s));
      const uint64_t r0 = uint64_t(h->row_ptr[s]), r1 = uint64_t(h->row_ptr[s + 1]);
      items.resize(r1 - r0);
      for (uint64_t e = r0; e < r1; ++e) {
        const uint32_t wbits = bf16 ? uint32_t(wb[e]) : [&] {
          uint32_t b;
          std::memcpy(&b, wf + e, 4);
          return b;
        }();
        items[e - r0] = RowItem{(uint64_t(tag[e]) << 32) | tgt_delay[e], wbits};
      }
      std::sort(items.begin(), items.end());
      uint32_t nl = 0, nv = 0;
      uint32_t last_tag = 0, last_node = 0xFFFFFFFFu;
      for (uint64_t e = r0; e < r1; ++e) {
        const RowItem& it = items[e - r0];
        const uint32_t tg = uint32_t(it.key >> 32);
        tgt_delay[e] = uint32_t(it.key);
        tag[e] = uint16_t(tg);
        if (bf16) wb[e] = uint16_t(it.w);
        else std::memcpy(wf + e, &it.w, 4);
        if (tg == 0) {
          ++nl;
        } else if (tg != last_tag) {
          ++nv;
          rc[tg - 1] += 1;
          const uint32_t node = (tg - 1) / G;
          if (node != last_node) {
            bc[node] += 1;
            last_node = node;
          }
          last_tag = tg;
        }
      }
      n_local[s] = nl;
      h->n_vp[s] = nv;
      // the own-partition part is sorted by delay: offsets of each delay's run
      if (nl > 0xFFFFu) __atomic_store_n(&too_long, 1, __ATOMIC_RELAXED);
      uint16_t* doff = delay_off + uint64_t(s) * (md + 1);
      uint32_t pos = 0;
      for (uint32_t d = 1; d <= md; ++d) {
        doff[d - 1] = uint16_t(pos);
        while (pos < nl && (tgt_delay[r0 + pos] >> 27) == d) ++pos;
      }
      doff[md] = uint16_t(nl);
    }
  }
  if (too_long)
    return fail(SNN_ERR_UNSUPPORTED, "a source has 65536 or more own-partition synapses");
  h->bucket_cap.assign(n_nodes, 0);
  h->recv_cap.assign(P, 0);
  for (int th = 0; th < h->threads; ++th) {
    for (uint32_t n = 0; n < n_nodes; ++n) h->bucket_cap[n] += bcap[th][n];
    for (uint32_t p = 0; p < P; ++p) h->recv_cap[p] += rcap[th][p];
  }
  h->pairs = 0;
  for (uint32_t s = 0; s < N; ++s) h->pairs += h->n_vp[s];
  h->bucket_total = 0;
  for (uint64_t c : h->bucket_cap) h->bucket_total += c;
  h->recv_total = 0;
  for (uint64_t c : h->recv_cap) h->recv_total += c;
  h->rows_done = true;
  return SNN_OK;
}

snn_status snn_setup_fill_routes(snn_setup_handle h, const uint32_t* tgt_delay,
                                 const void* weight, int64_t* vp_ptr, uint16_t* vp_part,
                                 uint64_t* vp_rec, int32_t* part_of_neuron,
                                 uint64_t* bucket_off, uint64_t* recv_off) {
  if (!h || !tgt_delay || !weight || !vp_ptr || !part_of_neuron || !bucket_off || !recv_off)
    return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  if (!h->rows_done) return fail(SNN_ERR_BAD_STATE, "snn_setup_fill_rows has not run");
  if (h->pairs && (!vp_part || !vp_rec)) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  const uint32_t N = h->N;
  vp_ptr[0] = 0;
  for (uint32_t s = 0; s < N; ++s) vp_ptr[s + 1] = vp_ptr[s] + h->n_vp[s];
  const uint16_t* tag = h->tag.data();
  const bool bf16 = h->spec.weight_type == SNN_W_BF16;
  const float* wf = static_cast<const float*>(weight);
  const uint16_t* wb = static_cast<const uint16_t*>(weight);
  int too_long = 0;
#pragma omp parallel for num_threads(h->threads) schedule(dynamic, 256)
  for (int64_t s = 0; s < int64_t(N); ++s) {
    const uint64_t r0 = uint64_t(h->row_ptr[s]), r1 = uint64_t(h->row_ptr[s + 1]);
    int64_t j = vp_ptr[s];
    uint16_t last = 0;
    uint64_t seg0 = 0;
    for (uint64_t e = r0; e <= r1; ++e) {
      const uint16_t tg = e < r1 ? tag[e] : 0;
      if (last != 0 && tg != last) {
        // close the segment of partition last - 1: [seg0, e)
        const uint64_t len = e - seg0;
        if (len >= (uint64_t(1) << 24)) __atomic_store_n(&too_long, 1, __ATOMIC_RELAXED);
        uint32_t wbits;
        if (bf16) wbits = wb[seg0];
        else std::memcpy(&wbits, wf + seg0, 4);
        vp_part[j] = uint16_t(last - 1);
        vp_rec[2 * j] = seg0 | (len << 40);
        vp_rec[2 * j + 1] = uint64_t(tgt_delay[seg0]) | (uint64_t(wbits) << 32);
        ++j;
      }
      if (tg != 0 && tg != last) seg0 = e;
      last = tg;
    }
  }
  if (too_long)
    return fail(SNN_ERR_UNSUPPORTED, "a source has 2^24 or more synapses into one partition");
  syn_part_map(h->gen, part_of_neuron);
  bucket_off[0] = 0;
  for (uint32_t n = 0; n < h->n_nodes; ++n) bucket_off[n + 1] = bucket_off[n] + h->bucket_cap[n];
  recv_off[0] = 0;
  for (uint32_t p = 0; p < h->P; ++p) recv_off[p + 1] = recv_off[p] + h->recv_cap[p];
  return SNN_OK;
}

void snn_setup_destroy(snn_setup_handle h) {
  if (!h) return;
  syn_destroy(h->gen);
  delete h;
}

snn_status snn_setup_model_params(const snn_model* m, snn_params* p) {
  if (!m || !p) return fail(SNN_ERR_INVALID_ARG, "NULL argument");
  if (!(m->dt_ms > 0) || !(m->tau_m_ms > 0))
    return fail(SNN_ERR_INVALID_ARG, "dt_ms and tau_m_ms must be positive");
  if (!(m->t_ref_ms >= 0) || !(m->nu_ext_hz >= 0) || !(m->rate_on_hz >= 0) ||
      !(m->rate_off_hz >= 0))
    return fail(SNN_ERR_INVALID_ARG, "t_ref_ms and the rates must be non-negative");
  const double steps_ref = std::nearbyint(m->t_ref_ms / m->dt_ms);
  if (steps_ref > 255) return fail(SNN_ERR_INVALID_ARG, "refractory period of %.0f steps > 255",
                                   steps_ref);
  const double lambda = m->nu_ext_hz * m->dt_ms * 1e-3;
  p->alpha = float(std::exp(-m->dt_ms / m->tau_m_ms));
  p->theta = float(m->theta_mv);
  p->u_reset = float(m->u_reset_mv);
  p->w_ext = float(m->w_ext_mv);
  p->n_ref = uint32_t(steps_ref);
  // floor(2^32 x), clamped to the uint32 range
  auto q32 = [](double x) -> uint32_t {
    const double v = std::floor(std::ldexp(x, 32));
    if (!(v > 0)) return 0u;
    return v >= 4294967295.0 ? 0xFFFFFFFFu : uint32_t(v);
  };
  double pmf = std::exp(-lambda), cdf = 0.0;
  for (int j = 0; j < 15; ++j) {
    if (j) pmf = pmf * lambda / j;
    cdf += pmf;
    p->poisson_thr[j] = q32(cdf);
  }
  p->raster_thr_on = q32(m->rate_on_hz * m->dt_ms * 1e-3);
  p->raster_thr_off = q32(m->rate_off_hz * m->dt_ms * 1e-3);
  return SNN_OK;
}

}  // extern "C"
