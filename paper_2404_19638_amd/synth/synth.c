/*
 * Seeded synthetic inputs for the local SDDMM/SpMM path.
 *
 * This file holds input tooling only: random number streams, R-MAT and
 * uniform-position sparsity patterns, block extraction, de-duplication,
 * caller-order shuffling and dense uniform matrices.  It contains none of
 * the method's arithmetic (no relabelling, no gathers, no products), and it
 * is shared by the oracle-side tests and the GPU path alike.
 *
 * Random numbers come from one counter-based generator: SplitMix64
 * (Steele, Lea and Flood, "Fast splittable pseudorandom number generators",
 * OOPSLA 2014), used as a keyed hash of (seed, counter).  Every draw is a pure
 * function of its counter, so every output is independent of the number of
 * OpenMP threads.
 *
 * R-MAT follows Chakrabarti, Zhan and Faloutsos (SDM 2004): each edge sample
 * descends `scale` levels, choosing one of four quadrants with probabilities
 * (a, b, c, d = 1-a-b-c), each quantised to a multiple of 2^-21.  Vertices are then relabelled by a seeded random
 * permutation, as the Graph500 generator does, so that blocks of a 2D grid
 * receive balanced shares.  Samples are de-duplicated (a sparse matrix stores
 * each (i,j) once) and finally shuffled into a seeded "caller order".
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define GOLDEN_GAMMA 0x9E3779B97F4A7C15ull

static inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Draw number `ctr` of the stream keyed by `seed`. */
uint64_t synth_draw(uint64_t seed, uint64_t ctr) {
  return mix64(mix64(seed) + (ctr + 1ull) * GOLDEN_GAMMA);
}

static inline uint64_t draw(uint64_t key, uint64_t ctr) {
  return mix64(key + (ctr + 1ull) * GOLDEN_GAMMA);
}

/* Uniform float in [-1,1): 24 random bits, exactly representable. */
static inline float sym24(uint64_t x) {
  return (float)((double)(int64_t)(x >> 40) * 0x1.0p-23 - 1.0);
}

/* Uniform integer in [0, n) by multiply-shift (Lemire 2019, without the
 * rejection step; the bias is below n / 2^64). */
static inline uint64_t below(uint64_t x, uint64_t n) {
  return (uint64_t)(((unsigned __int128)x * n) >> 64);
}

/* out[i] = U[-1,1) draw (ctr0 + i) of stream `seed`, for i < n. */
void synth_uniform_f32(uint64_t seed, uint64_t ctr0, int64_t n, float* out) {
  const uint64_t key = mix64(seed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = sym24(draw(key, ctr0 + (uint64_t)i));
}

/* Dense row-major block: out[r*ld + k] = U(seed, (row0 + r) * gcols + k) for
 * r < nrows, k < ncols.  Indexing by the global row keeps a matrix's values
 * independent of which block of it is materialised. */
void synth_dense_f32(uint64_t seed, int64_t row0, int64_t nrows, int64_t ncols,
                     int64_t gcols, int64_t ld, float* out) {
  const uint64_t key = mix64(seed);
#pragma omp parallel for schedule(static)
  for (int64_t r = 0; r < nrows; ++r) {
    const uint64_t base = (uint64_t)(row0 + r) * (uint64_t)gcols;
    for (int64_t k = 0; k < ncols; ++k) out[r * ld + k] = sym24(draw(key, base + (uint64_t)k));
  }
}

/* In-place seeded Fisher-Yates shuffle of [0, n) as a permutation. */
static void random_permutation(uint64_t key, int64_t n, int64_t* perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = i;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)below(draw(key, (uint64_t)i), (uint64_t)i + 1);
    int64_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
}

/* LSD radix sort of 64-bit keys (8-bit digits, only as many passes as the
 * key width needs).  Stable; tmp has n entries. */
static void radix_sort_u64(uint64_t* keys, uint64_t* tmp, int64_t n, int key_bits) {
  int passes = (key_bits + 7) / 8;
  uint64_t* src = keys; uint64_t* dst = tmp;
  int nth = omp_get_max_threads();
  int64_t* hist = (int64_t*)malloc(sizeof(int64_t) * 256 * (size_t)nth);
  for (int pass = 0; pass < passes; ++pass) {
    const int sh = 8 * pass;
    memset(hist, 0, sizeof(int64_t) * 256 * (size_t)nth);
#pragma omp parallel num_threads(nth)
    {
      int t = omp_get_thread_num();
      int64_t lo = n * t / nth, hi = n * (t + 1) / nth;
      int64_t* h = hist + 256 * t;
      for (int64_t i = lo; i < hi; ++i) h[(src[i] >> sh) & 255]++;
    }
    int64_t run = 0;
    for (int d = 0; d < 256; ++d)
      for (int t = 0; t < nth; ++t) { int64_t c = hist[256 * t + d]; hist[256 * t + d] = run; run += c; }
#pragma omp parallel num_threads(nth)
    {
      int t = omp_get_thread_num();
      int64_t lo = n * t / nth, hi = n * (t + 1) / nth;
      int64_t* h = hist + 256 * t;
      for (int64_t i = lo; i < hi; ++i) dst[h[(src[i] >> sh) & 255]++] = src[i];
    }
    uint64_t* s = src; src = dst; dst = s;
  }
  if (src != keys) memcpy(keys, src, sizeof(uint64_t) * (size_t)n);
  free(hist);
}

static int bits_for(int64_t range) {
  int b = 0;
  while (b < 63 && ((int64_t)1 << b) < range) ++b;
  return b;
}

/* Sort (row, col) keys, drop repeats, shuffle into caller order and split into
 * int64 row/col arrays.  Consumes `keys` (n entries, key = r << cb | c). */
static int64_t finish_pattern(uint64_t* keys, int64_t n, int rb, int cb, int64_t row_lo,
                              int64_t col_lo, uint64_t shuffle_key, int64_t** rows_out,
                              int64_t** cols_out) {
  uint64_t* tmp = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  radix_sort_u64(keys, tmp, n, rb + cb);
  int64_t m = 0;
  for (int64_t i = 0; i < n; ++i)
    if (i == 0 || keys[i] != keys[i - 1]) keys[m++] = keys[i];
  /* Caller order: a seeded Fisher-Yates shuffle of the distinct entries. */
  for (int64_t i = m - 1; i > 0; --i) {
    int64_t j = (int64_t)below(draw(shuffle_key, (uint64_t)i), (uint64_t)i + 1);
    uint64_t t = keys[i]; keys[i] = keys[j]; keys[j] = t;
  }
  int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
  int64_t* cols = (int64_t*)malloc(sizeof(int64_t) * (size_t)(m > 0 ? m : 1));
  const uint64_t cmask = (cb >= 64) ? ~0ull : ((1ull << cb) - 1ull);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) {
    rows[i] = row_lo + (int64_t)(keys[i] >> cb);
    cols[i] = col_lo + (int64_t)(keys[i] & cmask);
  }
  free(tmp);
  *rows_out = rows; *cols_out = cols;
  return m;
}

/*
 * R-MAT pattern restricted to the block [row_lo,row_hi) x [col_lo,col_hi).
 * nsamples edge samples are drawn over a 2^scale vertex set; with
 * `permute` != 0 every vertex id is relabelled by one seeded permutation.
 * Returns the number m of distinct entries kept and mallocs *rows / *cols
 * (global ids, caller order); release them with synth_free.
 */
int64_t synth_rmat_block(int scale, int64_t nsamples, double a, double b, double c,
                         uint64_t seed, int permute, int64_t row_lo, int64_t row_hi,
                         int64_t col_lo, int64_t col_hi, int64_t** rows_out,
                         int64_t** cols_out) {
  const uint64_t key_edges = mix64(seed ^ 0x52u);
  const uint64_t key_perm = mix64(seed ^ 0x50u);
  const uint64_t key_shuf = mix64(seed ^ 0x53u);
  const int64_t nv = (int64_t)1 << scale;
  int64_t* perm = NULL;
  if (permute) {
    perm = (int64_t*)malloc(sizeof(int64_t) * (size_t)nv);
    random_permutation(key_perm, nv, perm);
  }
  /* Membership bitmaps of the block's ranges in pre-permutation id space:
   * most samples are rejected with two cache-friendly bit tests instead of
   * two random reads of the permutation. */
  const int64_t nwords = (nv + 63) / 64;
  uint64_t* rsel = (uint64_t*)calloc((size_t)nwords, sizeof(uint64_t));
  uint64_t* csel = (uint64_t*)calloc((size_t)nwords, sizeof(uint64_t));
  for (int64_t v = 0; v < nv; ++v) {
    int64_t pv = perm ? perm[v] : v;
    if (pv >= row_lo && pv < row_hi) rsel[v >> 6] |= 1ull << (v & 63);
    if (pv >= col_lo && pv < col_hi) csel[v >> 6] |= 1ull << (v & 63);
  }
  const uint32_t t_a = (uint32_t)(a * 2097152.0 + 0.5);
  const uint32_t t_ab = (uint32_t)((a + b) * 2097152.0 + 0.5);
  const uint32_t t_abc = (uint32_t)((a + b + c) * 2097152.0 + 0.5);
  const int draws_per_edge = (scale + 2) / 3;
  const int rb = bits_for(row_hi - row_lo), cb = bits_for(col_hi - col_lo);
  int nth = omp_get_max_threads();
  int64_t* counts = (int64_t*)calloc((size_t)nth + 1, sizeof(int64_t));
  uint64_t** parts = (uint64_t**)calloc((size_t)nth, sizeof(uint64_t*));
#pragma omp parallel num_threads(nth)
  {
    int t = omp_get_thread_num();
    int64_t lo = nsamples * t / nth, hi = nsamples * (t + 1) / nth;
    int64_t cap = 1024, cnt = 0;
    uint64_t* buf = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)cap);
    for (int64_t e = lo; e < hi; ++e) {
      int64_t r = 0, col = 0;
      const uint64_t base = (uint64_t)e * (uint64_t)draws_per_edge;
      uint64_t x = 0;
      for (int l = 0; l < scale; ++l) {
        /* Three levels per 64-bit draw, each a 21-bit uniform u in
         * [0, 2^21) compared against the quadrant thresholds. */
        if (l % 3 == 0) x = draw(key_edges, base + (uint64_t)(l / 3));
        uint32_t u = (uint32_t)(x >> (64 - 21 * (l % 3 + 1))) & 0x1FFFFFu;
        int rbit = u >= t_ab;
        int cbit = (u >= t_a && u < t_ab) || u >= t_abc;
        r = (r << 1) | rbit;
        col = (col << 1) | cbit;
      }
      if (!((rsel[r >> 6] >> (r & 63)) & 1ull)) continue;
      if (!((csel[col >> 6] >> (col & 63)) & 1ull)) continue;
      if (perm) { r = perm[r]; col = perm[col]; }
      if (cnt == cap) { cap *= 2; buf = (uint64_t*)realloc(buf, sizeof(uint64_t) * (size_t)cap); }
      buf[cnt++] = ((uint64_t)(r - row_lo) << cb) | (uint64_t)(col - col_lo);
    }
    parts[t] = buf; counts[t + 1] = cnt;
  }
  for (int t = 0; t < nth; ++t) counts[t + 1] += counts[t];
  int64_t n = counts[nth];
  uint64_t* keys = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
  for (int t = 0; t < nth; ++t) {
    memcpy(keys + counts[t], parts[t], sizeof(uint64_t) * (size_t)(counts[t + 1] - counts[t]));
    free(parts[t]);
  }
  free(parts); free(counts); free(perm); free(rsel); free(csel);
  int64_t m = finish_pattern(keys, n, rb, cb, row_lo, col_lo, key_shuf, rows_out, cols_out);
  free(keys);
  return m;
}

/*
 * Exactly nnz distinct positions drawn uniformly from [0,nrows) x [0,ncols)
 * by rejection: positions are drawn in sequence and a repeat is skipped.
 * Caller order is draw order.  Offsets row_lo / col_lo turn local positions
 * into global ids.  Returns nnz (or -1 if nnz exceeds the number of cells).
 */
int64_t synth_uniform_block(int64_t nrows, int64_t ncols, int64_t nnz, uint64_t seed,
                            int64_t row_lo, int64_t col_lo, int64_t** rows_out,
                            int64_t** cols_out) {
  if ((double)nnz > (double)nrows * (double)ncols) return -1;
  const uint64_t key = mix64(seed ^ 0x55u);
  int64_t cap = 16;
  while (cap < 2 * nnz + 16) cap <<= 1;
  uint64_t* table = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)cap);
  memset(table, 0xff, sizeof(uint64_t) * (size_t)cap);
  int64_t* rows = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t* cols = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
  int64_t m = 0;
  uint64_t ctr = 0;
  while (m < nnz) {
    uint64_t x = draw(key, ctr++);
    int64_t r = (int64_t)below(x, (uint64_t)nrows);
    int64_t c = (int64_t)below(draw(key, ctr++), (uint64_t)ncols);
    uint64_t k = (uint64_t)r * (uint64_t)ncols + (uint64_t)c;
    uint64_t h = mix64(k) & (uint64_t)(cap - 1);
    int dup = 0;
    while (table[h] != ~0ull) {
      if (table[h] == k) { dup = 1; break; }
      h = (h + 1) & (uint64_t)(cap - 1);
    }
    if (dup) continue;
    table[h] = k;
    rows[m] = row_lo + r; cols[m] = col_lo + c; ++m;
  }
  free(table);
  *rows_out = rows; *cols_out = cols;
  return m;
}

void synth_free(void* p) { free(p); }

int synth_threads(void) { return omp_get_max_threads(); }

/* n raw 64-bit counter draws: out[i] = draw(seed, ctr0 + i) (random numbers a
 * method consumes, handed to both the GPU path and the oracle). */
void synth_draws_u64(uint64_t seed, uint64_t ctr0, int64_t n, uint64_t* out) {
  const uint64_t key = mix64(seed);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) out[i] = draw(key, ctr0 + (uint64_t)i);
}
