/*
 * A plain C client of libspc3d: no Python and no PyTorch.  It allocates device
 * memory with the HIP runtime, runs the whole local step through the C entry
 * points (setup, gather of A and B rows, SDDMM + SpMM in one pass,
 * scatter-reduce) on a small block with global ids, and checks every result
 * against the FP64 oracle's C functions (liboracle.so, test infrastructure):
 * the maps, CSR arrays, packed rows and the scatter-reduce bit for bit, the
 * SDDMM and SpMM values within 1e-5 of the magnitude sum of their terms.
 * The same pass with the scatter-reduce folded in must leave the slab bit for
 * bit as the separate scatter-reduce did, and the entry point without a
 * buffer argument must reproduce the buffered pass bit for bit.
 * It also exercises three error paths (an id outside the block's range, a
 * bad argument, a destroyed plan).  Exit status 0 and the line
 * "abi_client: ok" mean every check passed.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "spc3d.h"

/* The oracle's entry points used here (oracle/oracle.c). */
int oracle_relabel(int64_t nnz, const int64_t* row_gid, const int64_t* col_gid, int64_t row_lo,
                   int64_t row_hi, int64_t col_lo, int64_t col_hi, int64_t* R_out,
                   int64_t* C_out, int64_t* gmap_r, int64_t* gmap_c, int32_t* lmap_r,
                   int32_t* lmap_c, int32_t* rowptr, int32_t* colidx, int32_t* perm,
                   int32_t* colptr, int32_t* rowidx_t, int32_t* slot_t);
void oracle_gather_f32(int64_t n, const int64_t* gmap, int64_t lo, const float* src, int64_t ld,
                       int64_t k0, int64_t kz, float* packed);
void oracle_scatter_add_f32(int64_t n, const int64_t* gmap, int64_t lo, const float* packed,
                            int64_t kz, float* dst, int64_t ld, int64_t k0);
void oracle_sddmm(int64_t nnz, const int64_t* row_gid, const int64_t* col_gid, int64_t row_lo,
                  int64_t col_lo, const float* vals, const float* A, int64_t lda, const float* B,
                  int64_t ldb, int64_t k0, int64_t kz, double* out, double* mag);
void oracle_spmm(int64_t nnz, const int64_t* row_gid, const int64_t* col_gid, int64_t row_lo,
                 int64_t col_lo, const int32_t* lmap_r, int64_t R, const float* vals,
                 const float* B, int64_t ldb, int64_t k0, int64_t kz, double* Y, double* mag);

#define HIPCHECK(x)                                                              \
  do {                                                                           \
    hipError_t e_ = (x);                                                         \
    if (e_ != hipSuccess) {                                                      \
      fprintf(stderr, "%s failed: %s\n", #x, hipGetErrorString(e_));            \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

#define CHECK(x)                                                                 \
  do {                                                                           \
    spc3d_status s_ = (x);                                                       \
    if (s_ != SPC3D_OK) {                                                        \
      fprintf(stderr, "%s: %s (%s)\n", #x, spc3d_status_string(s_), spc3d_last_error()); \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

#define EXPECT(cond, ...)                                                        \
  do {                                                                           \
    if (!(cond)) {                                                               \
      fprintf(stderr, "check failed: " __VA_ARGS__);                             \
      fprintf(stderr, "\n");                                                     \
      return 1;                                                                  \
    }                                                                            \
  } while (0)

/* SplitMix64 (Steele, Lea and Flood, 2014): this client's own input stream. */
static uint64_t next_u64(uint64_t* s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
static float next_unit(uint64_t* s) {   /* U[-1, 1) with 24 random bits */
  return (float)((double)(next_u64(s) >> 40) / 8388608.0 - 1.0);
}

static void* dev_copy(const void* h, size_t bytes) {
  void* d = NULL;
  if (hipMalloc(&d, bytes ? bytes : 1) != hipSuccess) return NULL;
  if (bytes && hipMemcpy(d, h, bytes, hipMemcpyHostToDevice) != hipSuccess) return NULL;
  return d;
}

int main(void) {
  /* block: rows [1000, 1300), columns [5000, 5200); K = 64, slice [16, 48) */
  const int64_t row_lo = 1000, row_hi = 1300, col_lo = 5000, col_hi = 5200;
  const int64_t nr = row_hi - row_lo, nc = col_hi - col_lo, K = 64;
  const int32_t k0 = 16, kz = 32;
  const int64_t nnz = 2500;
  uint64_t seed = 2404;

  /* distinct positions, skewed toward low rows so that some rows are long and
   * some rows and columns stay empty */
  int64_t* row_gid = malloc(sizeof(int64_t) * nnz);
  int64_t* col_gid = malloc(sizeof(int64_t) * nnz);
  unsigned char* used = calloc((size_t)(nr * nc), 1);
  for (int64_t p = 0; p < nnz;) {
    uint64_t a = next_u64(&seed), b = next_u64(&seed);
    /* three entries in four fall in the first 32 rows */
    int64_t r = (int64_t)((a >> 11) % ((b >> 40) % 4 == 0 ? (uint64_t)nr : 32u));
    int64_t c = (int64_t)((b >> 11) % (uint64_t)(nc - 20));   /* the last 20 columns unused */
    if (used[r * nc + c]) continue;
    used[r * nc + c] = 1;
    row_gid[p] = row_lo + r;
    col_gid[p] = col_lo + c;
    ++p;
  }
  float* vals = malloc(sizeof(float) * nnz);
  for (int64_t p = 0; p < nnz; ++p) vals[p] = next_unit(&seed);
  float* A_src = malloc(sizeof(float) * nr * K);
  float* B_src = malloc(sizeof(float) * nc * K);
  float* Y_dst = malloc(sizeof(float) * nr * K);
  for (int64_t i = 0; i < nr * K; ++i) A_src[i] = next_unit(&seed);
  for (int64_t i = 0; i < nc * K; ++i) B_src[i] = next_unit(&seed);
  for (int64_t i = 0; i < nr * K; ++i) Y_dst[i] = next_unit(&seed);
  float* Y_dst0 = malloc(sizeof(float) * nr * K);   /* the slab before the step */
  memcpy(Y_dst0, Y_dst, sizeof(float) * nr * K);

  /* the oracle */
  int64_t R = 0, C = 0;
  int64_t* o_gmap_r = malloc(sizeof(int64_t) * nr);
  int64_t* o_gmap_c = malloc(sizeof(int64_t) * nc);
  int32_t* o_lmap_r = malloc(sizeof(int32_t) * nr);
  int32_t* o_lmap_c = malloc(sizeof(int32_t) * nc);
  int32_t* o_rowptr = malloc(sizeof(int32_t) * (nr + 1));
  int32_t* o_colidx = malloc(sizeof(int32_t) * nnz);
  int32_t* o_perm = malloc(sizeof(int32_t) * nnz);
  EXPECT(oracle_relabel(nnz, row_gid, col_gid, row_lo, row_hi, col_lo, col_hi, &R, &C, o_gmap_r,
                        o_gmap_c, o_lmap_r, o_lmap_c, o_rowptr, o_colidx, o_perm, NULL, NULL,
                        NULL) == 0,
         "oracle relabel");

  /* device inputs */
  hipStream_t st;
  HIPCHECK(hipStreamCreate(&st));
  int64_t* d_row = dev_copy(row_gid, sizeof(int64_t) * nnz);
  int64_t* d_col = dev_copy(col_gid, sizeof(int64_t) * nnz);
  float* d_vals_caller = dev_copy(vals, sizeof(float) * nnz);
  float* d_A_src = dev_copy(A_src, sizeof(float) * nr * K);
  float* d_B_src = dev_copy(B_src, sizeof(float) * nc * K);
  float* d_Y_dst = dev_copy(Y_dst, sizeof(float) * nr * K);
  EXPECT(d_row && d_col && d_vals_caller && d_A_src && d_B_src && d_Y_dst, "device inputs");

  /* setup */
  size_t ws_bytes = 0;
  CHECK(spc3d_plan_workspace_size(nnz, row_lo, row_hi, col_lo, col_hi, 0, &ws_bytes));
  void* d_ws = NULL;
  HIPCHECK(hipMalloc(&d_ws, ws_bytes));
  spc3d_plan plan = NULL;
  CHECK(spc3d_plan_create_coo(&plan, nnz, d_row, d_col, row_lo, row_hi, col_lo, col_hi, 0, d_ws,
                              ws_bytes, st));
  int64_t gR, gC, gnnz;
  CHECK(spc3d_plan_query(plan, &gR, &gC, &gnnz));
  EXPECT(gR == R && gC == C && gnnz == nnz, "R, C, nnz: %lld %lld %lld vs %lld %lld %lld",
         (long long)gR, (long long)gC, (long long)gnnz, (long long)R, (long long)C,
         (long long)nnz);
  spc3d_maps m;
  CHECK(spc3d_plan_maps(plan, &m));
  int64_t* g_gmap_r = malloc(sizeof(int64_t) * R);
  int64_t* g_gmap_c = malloc(sizeof(int64_t) * C);
  int32_t* g_rowptr = malloc(sizeof(int32_t) * (R + 1));
  int32_t* g_colidx = malloc(sizeof(int32_t) * nnz);
  int32_t* g_perm = malloc(sizeof(int32_t) * nnz);
  HIPCHECK(hipMemcpy(g_gmap_r, m.gmap_r, sizeof(int64_t) * R, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(g_gmap_c, m.gmap_c, sizeof(int64_t) * C, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(g_rowptr, m.rowptr, sizeof(int32_t) * (R + 1), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(g_colidx, m.colidx, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(g_perm, m.perm, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  EXPECT(!memcmp(g_gmap_r, o_gmap_r, sizeof(int64_t) * R), "gmap_r");
  EXPECT(!memcmp(g_gmap_c, o_gmap_c, sizeof(int64_t) * C), "gmap_c");
  EXPECT(!memcmp(g_rowptr, o_rowptr, sizeof(int32_t) * (R + 1)), "rowptr");
  EXPECT(!memcmp(g_colidx, o_colidx, sizeof(int32_t) * nnz), "colidx");
  EXPECT(!memcmp(g_perm, o_perm, sizeof(int32_t) * nnz), "perm");

  /* the step */
  float *d_A = NULL, *d_B = NULL, *d_vals = NULL, *d_out = NULL, *d_Y = NULL;
  HIPCHECK(hipMalloc((void**)&d_A, sizeof(float) * R * kz));
  HIPCHECK(hipMalloc((void**)&d_B, sizeof(float) * C * kz));
  HIPCHECK(hipMalloc((void**)&d_vals, sizeof(float) * nnz));
  HIPCHECK(hipMalloc((void**)&d_out, sizeof(float) * nnz));
  HIPCHECK(hipMalloc((void**)&d_Y, sizeof(float) * R * kz));
  size_t buf_bytes = 0;
  CHECK(spc3d_spmm_buffer_size(plan, 0, kz, -1, &buf_bytes));
  void* d_buf = NULL;
  HIPCHECK(hipMalloc(&d_buf, buf_bytes ? buf_bytes : 1));
  CHECK(spc3d_permute_values(plan, SPC3D_CALLER_TO_SLOT, d_vals_caller, d_vals, st));
  CHECK(spc3d_gather(plan, SPC3D_ROWS, d_A_src, SPC3D_F32, K, k0, kz, d_A, SPC3D_F32, st));
  CHECK(spc3d_gather(plan, SPC3D_COLS, d_B_src, SPC3D_F32, K, k0, kz, d_B, SPC3D_F32, st));
  CHECK(spc3d_sddmm_spmm(plan, d_vals, d_A, d_B, SPC3D_F32, kz, d_out, d_Y, SPC3D_OVERWRITE, -1,
                         d_buf, buf_bytes, st));
  CHECK(spc3d_scatter_reduce(plan, SPC3D_ROWS, d_Y, kz, d_Y_dst, K, k0, st));
  HIPCHECK(hipStreamSynchronize(st));

  float* A_loc = malloc(sizeof(float) * R * kz);
  float* B_loc = malloc(sizeof(float) * C * kz);
  float* out = malloc(sizeof(float) * nnz);
  float* Y = malloc(sizeof(float) * R * kz);
  float* Y_after = malloc(sizeof(float) * nr * K);
  HIPCHECK(hipMemcpy(A_loc, d_A, sizeof(float) * R * kz, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(B_loc, d_B, sizeof(float) * C * kz, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(out, d_out, sizeof(float) * nnz, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(Y, d_Y, sizeof(float) * R * kz, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(Y_after, d_Y_dst, sizeof(float) * nr * K, hipMemcpyDeviceToHost));

  /* packed rows: bit for bit */
  float* want_A = malloc(sizeof(float) * R * kz);
  float* want_B = malloc(sizeof(float) * C * kz);
  oracle_gather_f32(R, o_gmap_r, row_lo, A_src, K, k0, kz, want_A);
  oracle_gather_f32(C, o_gmap_c, col_lo, B_src, K, k0, kz, want_B);
  EXPECT(!memcmp(A_loc, want_A, sizeof(float) * R * kz), "packed A");
  EXPECT(!memcmp(B_loc, want_B, sizeof(float) * C * kz), "packed B");

  /* SDDMM (slot order on the GPU, caller order in the oracle) and SpMM */
  double* o_out = malloc(sizeof(double) * nnz);
  double* o_mag = malloc(sizeof(double) * nnz);
  oracle_sddmm(nnz, row_gid, col_gid, row_lo, col_lo, vals, A_src, K, B_src, K, k0, kz, o_out,
               o_mag);
  double worst = 0.0;
  for (int64_t s = 0; s < nnz; ++s) {
    const int64_t p = g_perm[s];
    const double err = fabs((double)out[s] - o_out[p]);
    EXPECT(err <= 1e-5 * o_mag[p], "SDDMM slot %lld: %.9g vs %.9g (M %.3g)", (long long)s,
           (double)out[s], o_out[p], o_mag[p]);
    if (o_mag[p] > 0 && err / o_mag[p] > worst) worst = err / o_mag[p];
  }
  double* o_Y = malloc(sizeof(double) * R * kz);
  double* o_Ymag = malloc(sizeof(double) * R * kz);
  oracle_spmm(nnz, row_gid, col_gid, row_lo, col_lo, o_lmap_r, R, vals, B_src, K, k0, kz, o_Y,
              o_Ymag);
  for (int64_t i = 0; i < R * kz; ++i) {
    const double err = fabs((double)Y[i] - o_Y[i]);
    EXPECT(err <= 1e-5 * o_Ymag[i], "SpMM element %lld: %.9g vs %.9g (M %.3g)", (long long)i,
           (double)Y[i], o_Y[i], o_Ymag[i]);
    if (o_Ymag[i] > 0 && err / o_Ymag[i] > worst) worst = err / o_Ymag[i];
  }

  /* scatter-reduce of the GPU's own Y: bit for bit, untouched rows unchanged */
  oracle_scatter_add_f32(R, o_gmap_r, row_lo, Y, kz, Y_dst, K, k0);
  EXPECT(!memcmp(Y_after, Y_dst, sizeof(float) * nr * K), "scatter-reduce");

  /* the scatter-reduce folded into the pass, on a fresh copy of the slab:
   * the same row sums added in the same order, so the same bits */
  float *d_Y_dst2 = dev_copy(Y_dst0, sizeof(float) * nr * K), *d_out2 = NULL;
  EXPECT(d_Y_dst2, "second slab");
  HIPCHECK(hipMalloc((void**)&d_out2, sizeof(float) * nnz));
  CHECK(spc3d_sddmm_spmm_scatter(plan, d_vals, d_A, d_B, SPC3D_F32, kz, d_out2, SPC3D_OVERWRITE,
                                 d_Y_dst2, K, k0, -1, d_buf, buf_bytes, st));
  HIPCHECK(hipStreamSynchronize(st));
  float* out2 = malloc(sizeof(float) * nnz);
  HIPCHECK(hipMemcpy(out2, d_out2, sizeof(float) * nnz, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(Y_after, d_Y_dst2, sizeof(float) * nr * K, hipMemcpyDeviceToHost));
  EXPECT(!memcmp(out2, out, sizeof(float) * nnz), "folded pass: SDDMM values");
  EXPECT(!memcmp(Y_after, Y_dst, sizeof(float) * nr * K), "folded pass: slab");

  /* the entry point that allocates nothing and takes no buffer */
  float* d_Y2 = NULL;
  HIPCHECK(hipMalloc((void**)&d_Y2, sizeof(float) * R * kz));
  CHECK(spc3d_sddmm_spmm_static(plan, d_vals, d_A, d_B, SPC3D_F32, kz, d_out2, d_Y2,
                                SPC3D_OVERWRITE, -1, st));
  HIPCHECK(hipStreamSynchronize(st));
  float* Y2 = malloc(sizeof(float) * R * kz);
  HIPCHECK(hipMemcpy(out2, d_out2, sizeof(float) * nnz, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(Y2, d_Y2, sizeof(float) * R * kz, hipMemcpyDeviceToHost));
  EXPECT(!memcmp(out2, out, sizeof(float) * nnz), "no-buffer pass: SDDMM values");
  EXPECT(!memcmp(Y2, Y, sizeof(float) * R * kz), "no-buffer pass: SpMM rows");
  hipFree(d_Y_dst2); hipFree(d_out2); hipFree(d_Y2);

  /* error paths */
  EXPECT(spc3d_gather(plan, SPC3D_ROWS, d_A_src, SPC3D_F32, K, k0, 0, d_A, SPC3D_F32, st) ==
             SPC3D_ERR_INVALID_ARG,
         "kz = 0 accepted");
  CHECK(spc3d_plan_destroy(plan));
  EXPECT(spc3d_plan_query(plan, &gR, &gC, &gnnz) == SPC3D_ERR_BAD_HANDLE,
         "destroyed plan accepted");
  row_gid[7] = row_hi;   /* one id past the range */
  HIPCHECK(hipMemcpy(d_row, row_gid, sizeof(int64_t) * nnz, hipMemcpyHostToDevice));
  spc3d_plan bad = NULL;
  EXPECT(spc3d_plan_create_coo(&bad, nnz, d_row, d_col, row_lo, row_hi, col_lo, col_hi, 0, d_ws,
                               ws_bytes, st) == SPC3D_ERR_OUT_OF_RANGE,
         "id outside the range accepted");

  printf("abi_client: R=%lld C=%lld nnz=%lld, worst |err|/M %.3g\n", (long long)R, (long long)C,
         (long long)nnz, worst);
  printf("abi_client: ok\n");
  hipFree(d_row); hipFree(d_col); hipFree(d_vals_caller); hipFree(d_A_src); hipFree(d_B_src);
  hipFree(d_Y_dst); hipFree(d_ws); hipFree(d_A); hipFree(d_B); hipFree(d_vals); hipFree(d_out);
  hipFree(d_Y); hipFree(d_buf);
  hipStreamDestroy(st);
  return 0;
}
