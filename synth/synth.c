/*
 * synth.c -- seeded synthetic inputs for the FasterTucker hot path.
 *
 * This module draws random numbers only: sparse coordinates, tensor values
 * and initial parameters.  It holds none of the method's arithmetic and is
 * shared, as plain arrays, by the FP64 oracle and the GPU library.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014).  Its i-th output is the
 * mixing function applied to seed + (i+1)*gamma, so it is counter based and
 * any draw can be recomputed from (stream, counter) alone.  Each logical
 * stream gets its own key, derived from the user seed and a stream id.
 *
 * Coordinates: per mode a truncated Zipf law P(k) ~ (k+1)^-s on k=0..I-1
 * (s=0 is uniform), sampled with Walker/Vose alias tables.  Draw d of the
 * sequence is the coordinate whose mode-n index comes from counter d of mode
 * n's stream.  A sparse tensor has distinct coordinates, so the output keeps
 * the first nnz distinct coordinates in draw order (never a truncated sorted
 * set, which would bias toward small indices).  The result does not depend
 * on the number of threads.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define SYN_OK 0
#define SYN_ERR_ARG 1
#define SYN_ERR_NOMEM 2
#define SYN_MAX_ORDER 16

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static const uint64_t GOLDEN_GAMMA = 0x9E3779B97F4A7C15ULL;

/* key of a logical stream: distinct (seed, stream) pairs give unrelated keys */
uint64_t synth_stream_key(uint64_t seed, uint64_t stream) {
  return mix64(seed ^ mix64(stream * 0xD1B54A32D192ED03ULL + 0x632BE59BD9B4E019ULL));
}
/* counter-th output of a SplitMix64 generator started at `key` */
uint64_t synth_draw(uint64_t key, uint64_t counter) {
  return mix64(key + (counter + 1) * GOLDEN_GAMMA);
}
static inline double u01_open0(uint64_t x) { /* (0, 1] with 53 bits */
  return ((x >> 11) + 1) * 0x1.0p-53;
}
static inline double u01(uint64_t x) { /* [0, 1) with 53 bits */
  return (x >> 11) * 0x1.0p-53;
}

/* Stream ids.  Coordinates of mode n use STREAM_COORD + n. */
enum { STREAM_COORD = 0x100, STREAM_VALUE = 0x200, STREAM_PARAM = 0x300 };

/* ---------------- alias tables (Vose) ---------------- */
typedef struct {
  int64_t n;
  uint32_t* thresh; /* accept column k when the 32-bit coin is < thresh[k] */
  int32_t* alias;
  int uniform;
} alias_t;

static void alias_free(alias_t* a) {
  free(a->thresh);
  free(a->alias);
  a->thresh = NULL;
  a->alias = NULL;
}

static int alias_build(alias_t* a, int64_t n, double s) {
  a->n = n;
  a->uniform = (s == 0.0);
  a->thresh = NULL;
  a->alias = NULL;
  if (a->uniform) return SYN_OK;
  double* p = (double*)malloc(sizeof(double) * n);
  int64_t* small = (int64_t*)malloc(sizeof(int64_t) * n);
  int64_t* large = (int64_t*)malloc(sizeof(int64_t) * n);
  a->thresh = (uint32_t*)malloc(sizeof(uint32_t) * n);
  a->alias = (int32_t*)malloc(sizeof(int32_t) * n);
  if (!p || !small || !large || !a->thresh || !a->alias) {
    free(p); free(small); free(large); alias_free(a);
    return SYN_ERR_NOMEM;
  }
  /* normalising constant summed smallest-first for accuracy */
  double z = 0.0;
  for (int64_t k = n - 1; k >= 0; --k) z += pow((double)(k + 1), -s);
  for (int64_t k = 0; k < n; ++k) p[k] = pow((double)(k + 1), -s) / z * (double)n;
  int64_t ns = 0, nl = 0;
  for (int64_t k = 0; k < n; ++k) {
    if (p[k] < 1.0) small[ns++] = k; else large[nl++] = k;
  }
  double* prob = p; /* reuse: prob[k] becomes the acceptance probability */
  while (ns > 0 && nl > 0) {
    int64_t l = small[--ns];
    int64_t g = large[--nl];
    a->alias[l] = (int32_t)g;
    /* prob[l] is final */
    double pl = prob[l];
    double t = pl * 4294967296.0;
    a->thresh[l] = (t >= 4294967295.0) ? 0xFFFFFFFFu : (uint32_t)t;
    prob[g] = (prob[g] + pl) - 1.0;
    if (prob[g] < 1.0) small[ns++] = g; else large[nl++] = g;
  }
  while (nl > 0) { int64_t g = large[--nl]; a->alias[g] = (int32_t)g; a->thresh[g] = 0xFFFFFFFFu; }
  while (ns > 0) { int64_t l = small[--ns]; a->alias[l] = (int32_t)l; a->thresh[l] = 0xFFFFFFFFu; }
  free(p);
  free(small);
  free(large);
  return SYN_OK;
}

static inline int32_t alias_sample(const alias_t* a, uint64_t x) {
  uint64_t hi = x >> 32;
  int64_t col = (int64_t)((hi * (uint64_t)a->n) >> 32);
  if (a->uniform) return (int32_t)col;
  uint32_t coin = (uint32_t)(x & 0xFFFFFFFFu);
  return coin < a->thresh[col] ? (int32_t)col : a->alias[col];
}

/* ---------------- coordinates ---------------- */
typedef struct {
  int order;
  uint64_t keys[SYN_MAX_ORDER];
  alias_t tab[SYN_MAX_ORDER];
} coord_gen_t;

static inline void coord_of(const coord_gen_t* g, uint64_t d, int32_t* c) {
  for (int n = 0; n < g->order; ++n) c[n] = alias_sample(&g->tab[n], synth_draw(g->keys[n], d));
}
static inline uint64_t coord_hash(const int32_t* c, int order) {
  uint64_t h = 0x2545F4914F6CDD1DULL;
  for (int n = 0; n < order; ++n) h = mix64(h ^ ((uint64_t)(uint32_t)c[n] + 0x9E3779B97F4A7C15ULL * (n + 1)));
  return h;
}

/*
 * synth_coords: first `nnz` distinct coordinates of the draw sequence.
 *   dims[order], zipf_s[order] (0 = uniform), coords_out[order][nnz] (SoA).
 *   draws_used (may be NULL) receives the number of draws consumed.
 * The hash table is split into P partitions by hash; one thread owns each
 * partition and scans the draws in order, so "first occurrence" is decided
 * in draw order whatever the thread count.
 */
int synth_coords(int order, const int64_t* dims, const double* zipf_s, int64_t nnz, uint64_t seed,
                 int32_t* coords_out, int64_t* draws_used) {
  if (order < 1 || order > SYN_MAX_ORDER || nnz < 0 || !dims || !zipf_s || (!coords_out && nnz > 0))
    return SYN_ERR_ARG;
  double space = 1.0;
  for (int n = 0; n < order; ++n) {
    if (dims[n] < 1 || dims[n] > 0x7FFFFFFF) return SYN_ERR_ARG;
    space *= (double)dims[n];
  }
  if ((double)nnz > space) return SYN_ERR_ARG;
  if (nnz == 0) { if (draws_used) *draws_used = 0; return SYN_OK; }

  coord_gen_t g;
  g.order = order;
  for (int n = 0; n < order; ++n) g.tab[n].thresh = NULL, g.tab[n].alias = NULL;
  int rc = SYN_OK;
  for (int n = 0; n < order && rc == SYN_OK; ++n) {
    g.keys[n] = synth_stream_key(seed, STREAM_COORD + (uint64_t)n);
    rc = alias_build(&g.tab[n], dims[n], zipf_s[n]);
  }
  if (rc != SYN_OK) { for (int n = 0; n < order; ++n) alias_free(&g.tab[n]); return rc; }

  int P = 1;
#ifdef _OPENMP
  P = omp_get_max_threads();
  if (P < 1) P = 1;
  if (P > 64) P = 64;
#endif
  const int64_t block = nnz < (1 << 22) ? (nnz + 1024) : (int64_t)1 << 23;
  /* table: capacity >= 2 * (nnz + block), split into P power-of-two parts */
  int64_t want = 2 * (nnz + block) / P + 1;
  int64_t part = 1024;
  while (part < want) part <<= 1;
  uint64_t* thash = (uint64_t*)malloc(sizeof(uint64_t) * part * P);
  int64_t* tdraw = (int64_t*)malloc(sizeof(int64_t) * part * P);
  int32_t* bc = (int32_t*)malloc(sizeof(int32_t) * block * order);
  uint64_t* bh = (uint64_t*)malloc(sizeof(uint64_t) * block);
  uint8_t* first = (uint8_t*)malloc(block);
  int64_t* tcount = (int64_t*)malloc(sizeof(int64_t) * (P + 1));
  if (!thash || !tdraw || !bc || !bh || !first || !tcount) {
    rc = SYN_ERR_NOMEM;
    goto done;
  }
  for (int64_t i = 0; i < part * P; ++i) tdraw[i] = -1;

  int64_t kept = 0, d0 = 0;
  while (kept < nnz) {
    /* 1. draw a block: coordinates and hashes */
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < block; ++b) {
      int32_t c[SYN_MAX_ORDER];
      coord_of(&g, (uint64_t)(d0 + b), c);
      for (int n = 0; n < order; ++n) bc[(int64_t)n * block + b] = c[n];
      bh[b] = coord_hash(c, order);
      first[b] = 0;
    }
    /* 2. partitioned insert, each partition scans the block in draw order */
#pragma omp parallel for schedule(static, 1)
    for (int p = 0; p < P; ++p) {
      uint64_t* hh = thash + (int64_t)p * part;
      int64_t* dd = tdraw + (int64_t)p * part;
      for (int64_t b = 0; b < block; ++b) {
        uint64_t h = bh[b];
        if ((int)(h % (uint64_t)P) != p) continue;
        int64_t slot = (int64_t)((h >> 20) & (uint64_t)(part - 1));
        for (;;) {
          if (dd[slot] < 0) {
            dd[slot] = d0 + b;
            hh[slot] = h;
            first[b] = 1;
            break;
          }
          if (hh[slot] == h) {
            int32_t c[SYN_MAX_ORDER];
            int same = 1;
            int64_t od = dd[slot];
            if (od >= d0) {
              for (int n = 0; n < order; ++n) c[n] = bc[(int64_t)n * block + (od - d0)];
            } else {
              coord_of(&g, (uint64_t)od, c);
            }
            for (int n = 0; n < order; ++n) same &= (c[n] == bc[(int64_t)n * block + b]);
            if (same) break;
          }
          slot = (slot + 1) & (part - 1);
        }
      }
    }
    /* 3. keep first occurrences in draw order, up to nnz */
    int T = P;
    int64_t per = (block + T - 1) / T;
#pragma omp parallel for schedule(static, 1)
    for (int t = 0; t < T; ++t) {
      int64_t lo = t * per, hi = lo + per < block ? lo + per : block, cnt = 0;
      for (int64_t b = lo; b < hi; ++b) cnt += first[b];
      tcount[t + 1] = cnt;
    }
    tcount[0] = 0;
    for (int t = 0; t < T; ++t) tcount[t + 1] += tcount[t];
#pragma omp parallel for schedule(static, 1)
    for (int t = 0; t < T; ++t) {
      int64_t lo = t * per, hi = lo + per < block ? lo + per : block;
      int64_t pos = kept + tcount[t];
      for (int64_t b = lo; b < hi && pos < nnz; ++b) {
        if (!first[b]) continue;
        for (int n = 0; n < order; ++n) coords_out[(int64_t)n * nnz + pos] = bc[(int64_t)n * block + b];
        ++pos;
      }
    }
    int64_t added = tcount[T];
    if (kept + added >= nnz) {
      /* find how many draws of this block were needed */
      int64_t need = nnz - kept, seen = 0, b = 0;
      for (; b < block; ++b) {
        seen += first[b];
        if (seen == need) break;
      }
      if (draws_used) *draws_used = d0 + b + 1;
      kept = nnz;
    } else {
      kept += added;
    }
    d0 += block;
  }
done:
  free(thash); free(tdraw); free(bc); free(bh); free(first); free(tcount);
  for (int n = 0; n < order; ++n) alias_free(&g.tab[n]);
  return rc;
}

/*
 * synth_values: value of the k-th kept coordinate comes from counter k of the
 * value stream, so values are independent of the coordinates.
 *   kind 0: uniform integers lo..hi (lo, hi integral)
 *   kind 1: normal(mean=lo, std=hi) clipped to [clip_lo, clip_hi]
 */
int synth_values(int64_t nnz, int kind, double lo, double hi, double clip_lo, double clip_hi, uint64_t seed,
                 float* out) {
  if (nnz < 0 || (nnz > 0 && !out) || (kind != 0 && kind != 1)) return SYN_ERR_ARG;
  uint64_t key = synth_stream_key(seed, STREAM_VALUE);
  if (kind == 0) {
    int64_t a = (int64_t)lo, b = (int64_t)hi;
    if ((double)a != lo || (double)b != hi || b < a) return SYN_ERR_ARG;
    uint64_t span = (uint64_t)(b - a + 1);
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nnz; ++k) {
      uint64_t x = synth_draw(key, (uint64_t)k);
      out[k] = (float)(a + (int64_t)(((x >> 32) * span) >> 32));
    }
  } else {
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < nnz; ++k) {
      double u1 = u01_open0(synth_draw(key, 2 * (uint64_t)k));
      double u2 = u01(synth_draw(key, 2 * (uint64_t)k + 1));
      double z = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
      double v = lo + hi * z;
      if (v < clip_lo) v = clip_lo;
      if (v > clip_hi) v = clip_hi;
      out[k] = (float)v;
    }
  }
  return SYN_OK;
}

/* synth_normal: count samples of N(mean, std^2) rounded to float, stream (STREAM_PARAM, tag). */
int synth_normal(int64_t count, double mean, double std, uint64_t seed, uint64_t tag, float* out) {
  if (count < 0 || (count > 0 && !out)) return SYN_ERR_ARG;
  uint64_t key = synth_stream_key(seed, STREAM_PARAM + tag * 0x10000ULL);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) {
    double u1 = u01_open0(synth_draw(key, 2 * (uint64_t)k));
    double u2 = u01(synth_draw(key, 2 * (uint64_t)k + 1));
    out[k] = (float)(mean + std * sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2));
  }
  return SYN_OK;
}

/* synth_uniform_index: count indices uniform on [0, n), stream (STREAM_PARAM, tag). */
int synth_uniform_index(int64_t count, int64_t n, uint64_t seed, uint64_t tag, int32_t* out) {
  if (count < 0 || n < 1 || n > 0x7FFFFFFF || (count > 0 && !out)) return SYN_ERR_ARG;
  uint64_t key = synth_stream_key(seed, STREAM_PARAM + tag * 0x10000ULL + 1);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < count; ++k) out[k] = (int32_t)(((synth_draw(key, (uint64_t)k) >> 32) * (uint64_t)n) >> 32);
  return SYN_OK;
}
