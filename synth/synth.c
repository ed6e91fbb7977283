/*
 * synth.c — seeded synthetic network generator (inputs only; see synth.h).
 */
#include "synth.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

enum {
  S_SRC = 1,    /* source draw, remote flag / cross-partition flag */
  S_ATTR = 2,   /* delay, virtual partition */
  S_W = 3,      /* weight jitter */
  S_INIT = 4,   /* initial membrane state */
  S_SET = 5,    /* per-source vp sets */
  S_SIZE = 6,   /* partition sizes */
  S_CLUSTER = 7 /* cluster of a neuron */
};

struct syn_gen {
  syn_spec spec;
  uint32_t* part_start; /* P+1 (MATERIALIZED, BATCHED, CLUSTERED) */
  int32_t* part_map;    /* N, explicit neuron -> partition map, or NULL */
  double* cross_frac;   /* P (BATCHED) */
  uint16_t* vp_sets;    /* n_neurons * vp_set_size (LOOPBACK_SETS) */
  /* CLUSTERED: members of each cluster, ascending, and each neuron's cluster
     and position among its cluster's members */
  uint32_t* cl_start;   /* n_clusters + 1 */
  uint32_t* cl_member;  /* N */
  uint32_t* cl_of;      /* N */
  uint32_t* cl_pos;     /* N */
};

/* SplitMix64 output function (Steele, Lea, Flood 2014). */
static inline uint64_t mix64(uint64_t z) {
  z += 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

uint64_t syn_hash(uint64_t seed, uint64_t stream, uint64_t a, uint64_t b) {
  uint64_t h = mix64(seed ^ (stream * 0xD1B54A32D192ED03ull));
  h = mix64(h ^ a);
  return mix64(h ^ (b * 0xABC98388FB8FAC03ull));
}

/* Multiply-shift range reduction of a 32-bit draw onto [0, n). */
static inline uint32_t range32(uint32_t r, uint32_t n) {
  return (uint32_t)(((uint64_t)r * (uint64_t)n) >> 32);
}

/* 24-bit uniform on [0, 1). */
static inline double unit24(uint64_t h) { return (double)(h >> 40) * 0x1p-24; }

static uint32_t find_part(const uint32_t* start, uint32_t n_part, uint32_t x) {
  uint32_t lo = 0, hi = n_part; /* invariant: start[lo] <= x < start[hi] */
  while (hi - lo > 1) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (start[mid] <= x) lo = mid; else hi = mid;
  }
  return lo;
}

syn_gen* syn_create(const syn_spec* spec, const uint32_t* part_start,
                    const double* cross_frac) {
  if (!spec || spec->n_neurons < 2 || spec->k_in == 0 || spec->max_delay == 0 ||
      spec->n_partitions == 0 || spec->n_partitions > 65536)
    return NULL;
  uint32_t P = spec->n_partitions;
  int need_parts = spec->topology == SYN_TOPO_MATERIALIZED ||
                   spec->topology == SYN_TOPO_BATCHED ||
                   spec->topology == SYN_TOPO_CLUSTERED;
  if (spec->topology > SYN_TOPO_CLUSTERED) return NULL;
  if (spec->topology == SYN_TOPO_CLUSTERED &&
      (spec->n_clusters == 0 || spec->n_clusters > spec->n_neurons ||
       !(spec->p_in >= 0.0 && spec->p_in <= 1.0)))
    return NULL;
  if (need_parts) {
    if (!part_start || part_start[0] != 0 || part_start[P] != spec->n_neurons)
      return NULL;
    for (uint32_t p = 0; p < P; ++p)
      if (part_start[p + 1] <= part_start[p]) return NULL;
  } else if (P < 2) {
    return NULL;
  }
  if (spec->topology == SYN_TOPO_BATCHED && !cross_frac) return NULL;
  if (spec->topology == SYN_TOPO_LOOPBACK_SETS &&
      (spec->vp_set_size == 0 || spec->vp_set_size > P - 1))
    return NULL;

  syn_gen* g = (syn_gen*)calloc(1, sizeof(syn_gen));
  if (!g) return NULL;
  g->spec = *spec;
  if (need_parts) {
    g->part_start = (uint32_t*)malloc(sizeof(uint32_t) * (P + 1));
    memcpy(g->part_start, part_start, sizeof(uint32_t) * (P + 1));
  }
  if (spec->topology == SYN_TOPO_BATCHED) {
    g->cross_frac = (double*)malloc(sizeof(double) * P);
    memcpy(g->cross_frac, cross_frac, sizeof(double) * P);
  }
  if (spec->topology == SYN_TOPO_CLUSTERED) {
    /* each neuron's cluster, then the members of each cluster (counting sort) */
    uint32_t N = spec->n_neurons, C = spec->n_clusters;
    g->cl_start = (uint32_t*)calloc((size_t)C + 1, sizeof(uint32_t));
    g->cl_member = (uint32_t*)malloc(sizeof(uint32_t) * N);
    g->cl_of = (uint32_t*)malloc(sizeof(uint32_t) * N);
    g->cl_pos = (uint32_t*)malloc(sizeof(uint32_t) * N);
    if (!g->cl_start || !g->cl_member || !g->cl_of || !g->cl_pos) { syn_destroy(g); return NULL; }
    for (uint32_t i = 0; i < N; ++i) {
      g->cl_of[i] = range32((uint32_t)(syn_hash(spec->seed, S_CLUSTER, i, 0) >> 32), C);
      g->cl_start[g->cl_of[i] + 1]++;
    }
    for (uint32_t c = 0; c < C; ++c) g->cl_start[c + 1] += g->cl_start[c];
    uint32_t* fill = (uint32_t*)calloc(C, sizeof(uint32_t));
    if (!fill) { syn_destroy(g); return NULL; }
    for (uint32_t i = 0; i < N; ++i) {
      uint32_t c = g->cl_of[i];
      g->cl_pos[i] = fill[c];
      g->cl_member[g->cl_start[c] + fill[c]++] = i;
    }
    free(fill);
  }
  if (spec->topology == SYN_TOPO_LOOPBACK_SETS) {
    /* Floyd's sampling of m distinct values from [1, P-1], keyed by source. */
    uint32_t m = spec->vp_set_size, N = spec->n_neurons, n = P - 1;
    g->vp_sets = (uint16_t*)malloc(sizeof(uint16_t) * (size_t)N * m);
    if (!g->vp_sets) { syn_destroy(g); return NULL; }
#pragma omp parallel
    {
      uint8_t* seen = (uint8_t*)calloc(P, 1);
#pragma omp for schedule(static)
      for (int64_t s = 0; s < (int64_t)N; ++s) {
        uint16_t* out = g->vp_sets + (size_t)s * m;
        uint32_t cnt = 0;
        for (uint32_t j = n - m + 1; j <= n; ++j) {
          uint64_t h = syn_hash(spec->seed, S_SET, (uint64_t)s, j);
          uint32_t r = 1 + range32((uint32_t)(h >> 32), j); /* in [1, j] */
          uint32_t pick = seen[r] ? j : r;
          seen[pick] = 1;
          out[cnt++] = (uint16_t)pick;
        }
        /* ascending order, and clear the marks */
        for (uint32_t v = 1, c = 0; v <= n && c < m; ++v)
          if (seen[v]) { out[c++] = (uint16_t)v; seen[v] = 0; }
      }
      free(seen);
    }
  }
  return g;
}

void syn_destroy(syn_gen* g) {
  if (!g) return;
  free(g->part_start);
  free(g->part_map);
  free(g->cl_start);
  free(g->cl_member);
  free(g->cl_of);
  free(g->cl_pos);
  free(g->cross_frac);
  free(g->vp_sets);
  free(g);
}

uint32_t syn_part_of(const syn_gen* g, uint32_t x) {
  if (g->part_map) return (uint32_t)g->part_map[x];
  if (!g->part_start) return 0;
  return find_part(g->part_start, g->spec.n_partitions, x);
}

int syn_set_part_map(syn_gen* g, const int32_t* part) {
  if (!part || (g->spec.topology != SYN_TOPO_MATERIALIZED &&
                g->spec.topology != SYN_TOPO_CLUSTERED))
    return -1;
  for (uint32_t i = 0; i < g->spec.n_neurons; ++i)
    if (part[i] < 0 || (uint32_t)part[i] >= g->spec.n_partitions) return -1;
  int32_t* m = (int32_t*)malloc(sizeof(int32_t) * g->spec.n_neurons);
  if (!m) return -1;
  memcpy(m, part, sizeof(int32_t) * g->spec.n_neurons);
  free(g->part_map);
  g->part_map = m;
  return 0;
}

uint32_t syn_cluster_of(const syn_gen* g, uint32_t x) { return g->cl_of ? g->cl_of[x] : 0; }

void syn_part_map(const syn_gen* g, int32_t* part) {
  uint32_t N = g->spec.n_neurons;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)N; ++i) part[i] = (int32_t)syn_part_of(g, (uint32_t)i);
}

int syn_vp_set(const syn_gen* g, uint32_t src, uint16_t* out) {
  if (!g->vp_sets) return 0;
  memcpy(out, g->vp_sets + (size_t)src * g->spec.vp_set_size,
         sizeof(uint16_t) * g->spec.vp_set_size);
  return 1;
}

void syn_edge(const syn_gen* g, uint32_t tgt, uint32_t k, uint32_t* src_out,
              uint32_t* delay_out, uint32_t* vp_out, float* w_out) {
  const syn_spec* s = &g->spec;
  const uint32_t N = s->n_neurons;
  uint64_t h1 = syn_hash(s->seed, S_SRC, tgt, k);
  uint64_t h2 = syn_hash(s->seed, S_ATTR, tgt, k);
  uint32_t hi1 = (uint32_t)(h1 >> 32), lo1 = (uint32_t)h1;
  uint32_t hi2 = (uint32_t)(h2 >> 32), lo2 = (uint32_t)h2;
  uint32_t src, vp;

  if (s->topology == SYN_TOPO_BATCHED) {
    uint32_t q = find_part(g->part_start, s->n_partitions, tgt);
    uint32_t q0 = g->part_start[q], qn = g->part_start[q + 1] - q0;
    int cross = (double)lo1 < g->cross_frac[q] * 4294967296.0;
    if (qn == 1) cross = 1;      /* no other source inside q */
    if (qn == N) cross = 0;      /* no source outside q */
    if (cross) {
      uint32_t r = range32(hi1, N - qn);
      src = r < q0 ? r : r + qn;
    } else {
      src = q0 + range32(hi1, qn - 1);
      if (src >= tgt) src++;
    }
    vp = q;
  } else if (s->topology == SYN_TOPO_CLUSTERED) {
    uint32_t c = g->cl_of[tgt], c0 = g->cl_start[c], cn = g->cl_start[c + 1] - c0;
    int inside = (double)lo1 < s->p_in * 4294967296.0 && cn > 1;
    if (inside) {   /* uniform over the cluster's other members */
      uint32_t r = range32(hi1, cn - 1);
      src = g->cl_member[c0 + (r < g->cl_pos[tgt] ? r : r + 1)];
    } else {
      src = range32(hi1, N - 1);
      if (src >= tgt) src++;
    }
    vp = syn_part_of(g, tgt);
  } else {
    src = range32(hi1, N - 1);
    if (src >= tgt) src++;
    if (s->topology == SYN_TOPO_MATERIALIZED) {
      vp = syn_part_of(g, tgt);
    } else {
      int remote = (double)lo1 < s->remote_frac * 4294967296.0;
      if (!remote) vp = 0;
      else if (s->topology == SYN_TOPO_LOOPBACK)
        vp = 1 + range32(hi2, s->n_partitions - 1);
      else
        vp = g->vp_sets[(size_t)src * s->vp_set_size + range32(hi2, s->vp_set_size)];
    }
  }
  double w = (src % 5 == 4) ? s->w_inh : s->w_exc;
  if (s->w_jitter != 0.0) {
    uint64_t h3 = syn_hash(s->seed, S_W, tgt, k);
    w = w * (1.0 + s->w_jitter * (unit24(h3) - 0.5));
  }
  *src_out = src;
  *delay_out = 1 + range32(lo2, s->max_delay);
  *vp_out = vp;
  *w_out = (float)w;
}

void syn_edges(const syn_gen* g, uint32_t tgt_lo, uint32_t tgt_hi,
               uint32_t* src, uint32_t* tgt, uint8_t* delay, uint16_t* vp,
               float* w) {
  const uint32_t K = g->spec.k_in;
#pragma omp parallel for schedule(static)
  for (int64_t t = tgt_lo; t < (int64_t)tgt_hi; ++t) {
    size_t base = (size_t)(t - tgt_lo) * K;
    for (uint32_t k = 0; k < K; ++k) {
      uint32_t s_, d_, v_;
      float w_;
      syn_edge(g, (uint32_t)t, k, &s_, &d_, &v_, &w_);
      if (src) src[base + k] = s_;
      if (tgt) tgt[base + k] = (uint32_t)t;
      if (delay) delay[base + k] = (uint8_t)d_;
      if (vp) vp[base + k] = (uint16_t)v_;
      if (w) w[base + k] = w_;
    }
  }
}

void syn_initial_u(uint64_t seed, double theta, uint32_t n, float* u) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < (int64_t)n; ++i)
    u[i] = (float)(theta * unit24(syn_hash(seed, S_INIT, (uint64_t)i, 0)));
}

void syn_lognormal_sizes(uint64_t seed, uint32_t n_part, double median,
                         double sigma_ln, uint32_t lo, uint32_t hi,
                         uint32_t* sizes) {
  for (uint32_t p = 0; p < n_part; ++p) {
    /* Box-Muller from two 53-bit uniforms in (0, 1] and [0, 1) */
    uint64_t h1 = syn_hash(seed, S_SIZE, p, 0), h2 = syn_hash(seed, S_SIZE, p, 1);
    double u1 = ((double)(h1 >> 11) + 1.0) * 0x1p-53;
    double u2 = (double)(h2 >> 11) * 0x1p-53;
    double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
    double x = median * exp(sigma_ln * z);
    if (x < lo) x = lo;
    if (x > hi) x = hi;
    sizes[p] = (uint32_t)llround(x);
  }
}

void syn_uniform_doubles(uint64_t seed, uint32_t stream, uint32_t n, double lo,
                         double hi, double* out) {
  for (uint32_t i = 0; i < n; ++i) {
    uint64_t h = syn_hash(seed, 64 + stream, i, 0);
    out[i] = lo + (hi - lo) * ((double)(h >> 11) * 0x1p-53);
  }
}
