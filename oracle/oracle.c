/*
 * FP64 CPU oracle for the local SDDMM / SpMM path of SpComm3D
 * (Abubaker and Hoefler, "SpComm3D: A Framework for Enabling Sparse
 * Communication in 3D Sparse Kernels").
 *
 * TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct loops in double
 * precision, compiled without fast-math and without FP contraction.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark may load
 * this library; the product path never does.  It shares no code, header,
 * table or helper with the HIP library.
 *
 * Every function follows a definition from the paper:
 *   - localization of a sparse block (Section "Data distribution"): local ids
 *     are the ranks of the distinct global ids, empty rows/columns removed,
 *     with globalMap (local -> global) and localMap (global -> local);
 *   - SpC-BB packing and unpacking (Section "Sparse communication model",
 *     Method 1): copy the data unit of each global id into / out of a buffer;
 *   - SDDMM, Eq. (1): c_ij = s_ij * <a_i, b_j> for every stored (i,j);
 *   - SpMM, Eq. (2): a_i = sum_j s_ij * b_j;
 *   - the 3D split (Section "Sparsity-agnostic parallel algorithms", 3D
 *     paragraph, and the Compute phase of Section "Building 3D SDDMM and SpMM
 *     Algorithms"): each of Z instances works on K/Z columns of the dense
 *     matrices and partial results are summed.
 * Readings where the paper is silent are stated at each function.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------- relabel */

static int cmp_i64(const void* x, const void* y) {
  int64_t a = *(const int64_t*)x, b = *(const int64_t*)y;
  return (a > b) - (a < b);
}

typedef struct { int64_t major, minor, idx; } triple;

static int cmp_triple(const void* x, const void* y) {
  const triple* a = (const triple*)x;
  const triple* b = (const triple*)y;
  if (a->major != b->major) return (a->major > b->major) - (a->major < b->major);
  if (a->minor != b->minor) return (a->minor > b->minor) - (a->minor < b->minor);
  return (a->idx > b->idx) - (a->idx < b->idx);
}

/* globalMap = the distinct ids in ascending order; localMap[g - lo] = rank of
 * g, or -1 when g does not occur.  Returns the number of distinct ids. */
static int64_t localize_axis(int64_t nnz, const int64_t* gid, int64_t lo, int64_t hi,
                             int64_t* gmap, int32_t* lmap) {
  int64_t* s = (int64_t*)malloc(sizeof(int64_t) * (size_t)(nnz > 0 ? nnz : 1));
  memcpy(s, gid, sizeof(int64_t) * (size_t)nnz);
  qsort(s, (size_t)nnz, sizeof(int64_t), cmp_i64);
  int64_t n = 0;
  for (int64_t p = 0; p < nnz; ++p)
    if (p == 0 || s[p] != s[p - 1]) gmap[n++] = s[p];
  free(s);
  for (int64_t g = 0; g < hi - lo; ++g) lmap[g] = -1;
  for (int64_t l = 0; l < n; ++l) lmap[gmap[l] - lo] = (int32_t)l;
  return n;
}

/*
 * Localize one block S^z_{x,y} given in COO with global ids (caller order).
 * Outputs (caller-allocated):
 *   gmap_r[R], gmap_c[C] (capacity min(nnz, range)), lmap_r[row_hi-row_lo],
 *   lmap_c[col_hi-col_lo], rowptr[R+1], colidx[nnz], perm[nnz];
 *   when colptr != NULL also the column-major view colptr[C+1],
 *   rowidx_t[nnz] (local row of each column-major slot) and slot_t[nnz]
 *   (row-major slot of each column-major slot).
 * Row-major slots are ordered by (local row, local column, caller index), the
 * column-major ones by (local column, local row, caller index); perm maps a
 * row-major slot to its caller index.
 * Returns 0, or -1 when an id lies outside its range (outputs undefined).
 */
/* Owner-grouped local order (Method 2, SpC-SB/SpC-RB, of Section "Sparse
 * communication model": local data stored as the concatenation of the data
 * units exchanged with each peer, so a message lands in one contiguous
 * piece).  Given a group key per global id, local ids are re-assigned in
 * order of (key, global id); the maps are rewritten to match.  Returns -1 if
 * a used id has a key outside [0, ngroups). */
static int group_axis(int64_t n, int64_t lo, const int32_t* group, int32_t ngroups,
                      int64_t* gmap, int32_t* lmap) {
  triple* t = (triple*)malloc(sizeof(triple) * (size_t)(n > 0 ? n : 1));
  for (int64_t l = 0; l < n; ++l) {
    const int32_t k = group[gmap[l] - lo];
    if (k < 0 || k >= ngroups) {
      free(t);
      return -1;
    }
    t[l].major = k;
    t[l].minor = gmap[l];
    t[l].idx = l;
  }
  qsort(t, (size_t)n, sizeof(triple), cmp_triple);
  for (int64_t j = 0; j < n; ++j) {
    gmap[j] = t[j].minor;
    lmap[gmap[j] - lo] = (int32_t)j;
  }
  free(t);
  return 0;
}

int oracle_relabel_grouped(int64_t nnz, const int64_t* row_gid, const int64_t* col_gid,
                           int64_t row_lo, int64_t row_hi, int64_t col_lo, int64_t col_hi,
                           const int32_t* group_r, int32_t ngroups_r, const int32_t* group_c,
                           int32_t ngroups_c, int64_t* R_out, int64_t* C_out, int64_t* gmap_r,
                           int64_t* gmap_c, int32_t* lmap_r, int32_t* lmap_c, int32_t* rowptr,
                           int32_t* colidx, int32_t* perm, int32_t* colptr, int32_t* rowidx_t,
                           int32_t* slot_t) {
  for (int64_t p = 0; p < nnz; ++p) {
    if (row_gid[p] < row_lo || row_gid[p] >= row_hi) return -1;
    if (col_gid[p] < col_lo || col_gid[p] >= col_hi) return -1;
  }
  int64_t R = localize_axis(nnz, row_gid, row_lo, row_hi, gmap_r, lmap_r);
  int64_t C = localize_axis(nnz, col_gid, col_lo, col_hi, gmap_c, lmap_c);
  if (group_r && group_axis(R, row_lo, group_r, ngroups_r, gmap_r, lmap_r)) return -2;
  if (group_c && group_axis(C, col_lo, group_c, ngroups_c, gmap_c, lmap_c)) return -2;
  *R_out = R; *C_out = C;

  triple* t = (triple*)malloc(sizeof(triple) * (size_t)(nnz > 0 ? nnz : 1));
  for (int64_t p = 0; p < nnz; ++p) {
    t[p].major = lmap_r[row_gid[p] - row_lo];
    t[p].minor = lmap_c[col_gid[p] - col_lo];
    t[p].idx = p;
  }
  qsort(t, (size_t)nnz, sizeof(triple), cmp_triple);
  for (int64_t r = 0; r <= R; ++r) rowptr[r] = 0;
  for (int64_t q = 0; q < nnz; ++q) {
    rowptr[t[q].major + 1]++;
    colidx[q] = (int32_t)t[q].minor;
    perm[q] = (int32_t)t[q].idx;
  }
  for (int64_t r = 0; r < R; ++r) rowptr[r + 1] += rowptr[r];

  if (colptr) {
    int32_t* slot_of = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nnz > 0 ? nnz : 1));
    for (int64_t q = 0; q < nnz; ++q) slot_of[t[q].idx] = (int32_t)q;
    for (int64_t p = 0; p < nnz; ++p) {
      t[p].major = lmap_c[col_gid[p] - col_lo];
      t[p].minor = lmap_r[row_gid[p] - row_lo];
      t[p].idx = p;
    }
    qsort(t, (size_t)nnz, sizeof(triple), cmp_triple);
    for (int64_t c = 0; c <= C; ++c) colptr[c] = 0;
    for (int64_t q = 0; q < nnz; ++q) {
      colptr[t[q].major + 1]++;
      rowidx_t[q] = (int32_t)t[q].minor;
      slot_t[q] = slot_of[t[q].idx];
    }
    for (int64_t c = 0; c < C; ++c) colptr[c + 1] += colptr[c];
    free(slot_of);
  }
  free(t);
  return 0;
}

int oracle_relabel(int64_t nnz, const int64_t* row_gid, const int64_t* col_gid,
                   int64_t row_lo, int64_t row_hi, int64_t col_lo, int64_t col_hi,
                   int64_t* R_out, int64_t* C_out, int64_t* gmap_r, int64_t* gmap_c,
                   int32_t* lmap_r, int32_t* lmap_c, int32_t* rowptr, int32_t* colidx,
                   int32_t* perm, int32_t* colptr, int32_t* rowidx_t, int32_t* slot_t) {
  return oracle_relabel_grouped(nnz, row_gid, col_gid, row_lo, row_hi, col_lo, col_hi, NULL, 0,
                                NULL, 0, R_out, C_out, gmap_r, gmap_c, lmap_r, lmap_c, rowptr,
                                colidx, perm, colptr, rowidx_t, slot_t);
}

/* ------------------------------------------------------- pack / unpack */

/* SpC-BB packing: packed[l*kz + k] = src[(gmap[l]-lo)*ld + k0 + k]. */
void oracle_gather_f32(int64_t n, const int64_t* gmap, int64_t lo, const float* src, int64_t ld,
                       int64_t k0, int64_t kz, float* packed) {
  for (int64_t l = 0; l < n; ++l)
    for (int64_t k = 0; k < kz; ++k) packed[l * kz + k] = src[(gmap[l] - lo) * ld + k0 + k];
}

/*
 * FP32 -> bfloat16, round to nearest, ties to even, written from the
 * definition of the format: bfloat16 keeps the FP32 exponent range and 8
 * significant bits.  The result is the representable value nearest to x;
 * on a tie the one whose last significant bit is 0.  Magnitudes that round
 * beyond the largest finite value become infinity; NaN stays NaN (quiet,
 * sign kept); zeros and infinities are unchanged.  Returns the 16-bit
 * pattern, i.e. the upper half of the FP32 pattern of the rounded value.
 */
uint16_t oracle_bf16_rne(float xf) {
  uint32_t bits;
  memcpy(&bits, &xf, 4);
  if (isnan(xf)) return (uint16_t)((bits >> 16) | 0x0040u);
  if (isinf(xf) || xf == 0.0f) return (uint16_t)(bits >> 16);
  double x = (double)xf, a = fabs(x);
  int E;
  frexp(a, &E);                          /* a = m * 2^E, m in [0.5, 1) */
  int e = E < -125 ? -125 : E;           /* below 2^-126 the spacing stops shrinking */
  double ulp = ldexp(1.0, e - 8);        /* spacing of bfloat16 values near a */
  double q = floor(a / ulp);             /* exact: a / ulp is a scaled float */
  double lo = q * ulp, hi = (q + 1.0) * ulp;
  double pick;
  if (a - lo < hi - a) pick = lo;
  else if (hi - a < a - lo) pick = hi;
  else pick = (fmod(q, 2.0) == 0.0) ? lo : hi;
  float r = (float)(x < 0 ? -pick : pick);  /* exact unless it overflows to inf */
  if (pick >= ldexp(1.0, 128)) r = x < 0 ? -INFINITY : INFINITY;
  uint32_t rb;
  memcpy(&rb, &r, 4);
  return (uint16_t)(rb >> 16);
}

void oracle_bf16_rne_array(int64_t n, const float* x, uint16_t* out) {
  for (int64_t i = 0; i < n; ++i) out[i] = oracle_bf16_rne(x[i]);
}

/* Packing with conversion to bfloat16 on the way. */
void oracle_gather_bf16(int64_t n, const int64_t* gmap, int64_t lo, const float* src, int64_t ld,
                        int64_t k0, int64_t kz, uint16_t* packed) {
  for (int64_t l = 0; l < n; ++l)
    for (int64_t k = 0; k < kz; ++k)
      packed[l * kz + k] = oracle_bf16_rne(src[(gmap[l] - lo) * ld + k0 + k]);
}

/* SpC-BB unpacking with reduction (the SpMM PostComm received at the owner):
 * dst[(gmap[l]-lo)*ld + k0 + k] += packed[l*kz + k] in IEEE binary32. */
void oracle_scatter_add_f32(int64_t n, const int64_t* gmap, int64_t lo, const float* packed,
                            int64_t kz, float* dst, int64_t ld, int64_t k0) {
  for (int64_t l = 0; l < n; ++l)
    for (int64_t k = 0; k < kz; ++k) {
      float* d = &dst[(gmap[l] - lo) * ld + k0 + k];
      *d = *d + packed[l * kz + k];
    }
}

/* ------------------------------------------------------------ compute */

/*
 * SDDMM, Eq. (1), straight from the global view of the local block: for every
 * stored entry p (caller order),
 *   out[p] = s_p * sum_{k<kz} A[(row_gid[p]-row_lo)*lda + k0 + k]
 *                            * B[(col_gid[p]-col_lo)*ldb + k0 + k],
 * summed in ascending k in double precision.  vals == NULL means s == 1
 * (pattern-only sampling).  mag[p] = |s_p| * sum_k |a_k b_k| bounds the
 * rounding error of any FP32 evaluation order.  A stored entry whose value is
 * zero is still a task (the pattern, not the values, defines the tasks).
 */
void oracle_sddmm(int64_t nnz, const int64_t* row_gid, const int64_t* col_gid, int64_t row_lo,
                  int64_t col_lo, const float* vals, const float* A, int64_t lda, const float* B,
                  int64_t ldb, int64_t k0, int64_t kz, double* out, double* mag) {
  for (int64_t p = 0; p < nnz; ++p) {
    const float* a = A + (row_gid[p] - row_lo) * lda + k0;
    const float* b = B + (col_gid[p] - col_lo) * ldb + k0;
    double dot = 0.0, m = 0.0;
    for (int64_t k = 0; k < kz; ++k) {
      double t = (double)a[k] * (double)b[k];
      dot += t;
      m += fabs(t);
    }
    double s = vals ? (double)vals[p] : 1.0;
    out[p] = s * dot;
    if (mag) mag[p] = fabs(s) * m;
  }
}

/*
 * SpMM, Eq. (2), for the rows of a localized block: with local ids
 * lr_p = lmap_r[row_gid[p]-row_lo],
 *   Y[lr][k] = sum_{p : lr_p = lr} s_p * B[(col_gid[p]-col_lo)*ldb + k0 + k]
 * accumulated over p in caller order, in double.  Y and mag are [R x kz],
 * zeroed here; mag holds the sum of |s_p b_k|.
 */
void oracle_spmm(int64_t nnz, const int64_t* row_gid, const int64_t* col_gid, int64_t row_lo,
                 int64_t col_lo, const int32_t* lmap_r, int64_t R, const float* vals,
                 const float* B, int64_t ldb, int64_t k0, int64_t kz, double* Y, double* mag) {
  for (int64_t i = 0; i < R * kz; ++i) { Y[i] = 0.0; if (mag) mag[i] = 0.0; }
  for (int64_t p = 0; p < nnz; ++p) {
    int64_t lr = lmap_r[row_gid[p] - row_lo];
    const float* b = B + (col_gid[p] - col_lo) * ldb + k0;
    double s = vals ? (double)vals[p] : 1.0;
    for (int64_t k = 0; k < kz; ++k) {
      double t = s * (double)b[k];
      Y[lr * kz + k] += t;
      if (mag) mag[lr * kz + k] += fabs(t);
    }
  }
}

/* ------------------------------------------------------ graph attention */

/*
 * Masked attention over a localized block (row-major slots rowptr/colidx):
 *   e_p     = <q_{r(p)}, k_{c(p)}>                (pattern-only SDDMM)
 *   alpha_p = exp(e_p - max_row) / sum_row exp(e - max_row)
 *   out_r   = sum_{p in row r} alpha_p v_{c(p)}   (SpMM with alpha)
 * Q is [R x K], Kf and V are [C x K], all double.  alpha, e are per slot.
 */
void oracle_attention_fwd(int64_t R, const int32_t* rowptr, const int32_t* colidx, int64_t K,
                          const double* Q, const double* Kf, const double* V, double* e,
                          double* alpha, double* out) {
  for (int64_t r = 0; r < R; ++r) {
    double mx = -INFINITY;
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
      double d = 0.0;
      for (int64_t k = 0; k < K; ++k) d += Q[r * K + k] * Kf[(int64_t)colidx[p] * K + k];
      e[p] = d;
      if (d > mx) mx = d;
    }
    double sum = 0.0;
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) sum += exp(e[p] - mx);
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) alpha[p] = exp(e[p] - mx) / sum;
    for (int64_t k = 0; k < K; ++k) out[r * K + k] = 0.0;
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p)
      for (int64_t k = 0; k < K; ++k) out[r * K + k] += alpha[p] * V[(int64_t)colidx[p] * K + k];
  }
}

/*
 * Gradients of the attention above for an upstream gradient dout [R x K],
 * written from the chain rule entry by entry:
 *   dalpha_p = <dout_{r(p)}, v_{c(p)}>
 *   de_p     = alpha_p * (dalpha_p - sum_{p' in row} alpha_p' dalpha_p')
 *   dQ_r     = sum_{p in row r} de_p k_{c(p)}
 *   dKf_c    = sum_{p in column c} de_p q_{r(p)}
 *   dV_c     = sum_{p in column c} alpha_p dout_{r(p)}
 * dQ [R x K], dKf and dV [C x K] are zeroed here; de has one entry per slot.
 */
void oracle_attention_bwd(int64_t R, int64_t C, const int32_t* rowptr, const int32_t* colidx,
                          int64_t K, const double* Q, const double* Kf, const double* V,
                          const double* alpha, const double* dout, double* de, double* dQ,
                          double* dKf, double* dV) {
  for (int64_t i = 0; i < R * K; ++i) dQ[i] = 0.0;
  for (int64_t i = 0; i < C * K; ++i) { dKf[i] = 0.0; dV[i] = 0.0; }
  for (int64_t r = 0; r < R; ++r) {
    double acc = 0.0;
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
      double da = 0.0;
      for (int64_t k = 0; k < K; ++k) da += dout[r * K + k] * V[(int64_t)colidx[p] * K + k];
      de[p] = da;                       /* holds dalpha until the row sum is known */
      acc += alpha[p] * da;
    }
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) de[p] = alpha[p] * (de[p] - acc);
    for (int32_t p = rowptr[r]; p < rowptr[r + 1]; ++p) {
      int64_t c = colidx[p];
      for (int64_t k = 0; k < K; ++k) {
        dQ[r * K + k] += de[p] * Kf[c * K + k];
        dKf[c * K + k] += de[p] * Q[r * K + k];
        dV[c * K + k] += alpha[p] * dout[r * K + k];
      }
    }
  }
}

/* ------------------------------------------ lambda and Algorithm 1 owners */

/* One block row of a Dist3D grid (Section "Sparsity-aware Communication
 * Analysis of 3D SDDMM"): part p uses the counts[p] ids gmaps[p][..] of
 * [lo, hi).  lambda[i-lo] = number of parts using i.  Algorithm 1 gives i to
 * a uniformly random part among those that use it; with the 64-bit draw r of
 * the id, the pick is the candidate of rank floor(r * lambda / 2^64) in
 * ascending part order (rank 0 without draws): a reading of "pick a random
 * p in candidates" for a given uniform draw.  owned[p] counts the ids part p
 * owns; comm[p*nparts + q] counts the ids part p uses and part q != p owns
 * (rows p receives from q).  Brute force over a dense use matrix. */
void oracle_lambda_owners(int nparts, const int64_t* const* gmaps, const int64_t* counts,
                          int64_t lo, int64_t hi, const uint64_t* rnd, int32_t* lambda,
                          int32_t* owner, int64_t* owned, int64_t* comm) {
  const int64_t n = hi - lo;
  unsigned char* uses = (unsigned char*)calloc((size_t)(n > 0 ? n : 1) * (size_t)nparts, 1);
  for (int p = 0; p < nparts; ++p)
    for (int64_t l = 0; l < counts[p]; ++l) uses[(gmaps[p][l] - lo) * nparts + p] = 1;
  for (int p = 0; p < nparts; ++p) owned[p] = 0;
  for (int64_t q = 0; q < (int64_t)nparts * nparts; ++q) comm[q] = 0;
  for (int64_t i = 0; i < n; ++i) {
    int lam = 0;
    for (int p = 0; p < nparts; ++p) lam += uses[i * nparts + p];
    lambda[i] = lam;
    owner[i] = -1;
    if (lam == 0) continue;
    const uint64_t k = rnd ? (uint64_t)(((unsigned __int128)rnd[i] * (uint64_t)lam) >> 64) : 0;
    uint64_t seen = 0;
    for (int p = 0; p < nparts; ++p) {
      if (!uses[i * nparts + p]) continue;
      if (seen == k) {
        owner[i] = p;
        break;
      }
      ++seen;
    }
    owned[owner[i]] += 1;
  }
  for (int p = 0; p < nparts; ++p)
    for (int64_t l = 0; l < counts[p]; ++l) {
      const int q = owner[gmaps[p][l] - lo];
      if (q != p) comm[(int64_t)p * nparts + q] += 1;
    }
  free(uses);
}
