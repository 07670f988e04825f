/*
 * spc3d — the local data-parallel hot path of 3D sparsity-aware SDDMM and
 * SpMM (SpComm3D, Abubaker and Hoefler) on one AMD Instinct MI355X (gfx950).
 *
 * One GPU plays one processor P_{x,y,z} of the paper's 3D grid.  Its work per
 * iteration is the local part of the three phases the paper defines for every
 * sparse kernel (Section "The SpComm3D Framework", General structure):
 *
 *   setup (once per sparsity pattern)   spc3d_plan_create_coo
 *       localization of the block S_{x,y}: compact local row/column ids with
 *       globalMap / localMap, empty rows and columns removed
 *       (Section "Data distribution");
 *   PreComm, local side                 spc3d_gather
 *       pack the dense data units (row slices of A and B over the K-slice)
 *       that the block's nonzeros touch, SpC-BB style (Section "Sparse
 *       communication model", Method 1);
 *   Compute                             spc3d_sddmm, spc3d_spmm
 *       Eq. (1) and Eq. (2) over the localized block with the K/Z slice
 *       (Section "Building 3D SDDMM and SpMM Algorithms", The Compute phase);
 *   PostComm, local side                spc3d_scatter_reduce, and the
 *       ACCUMULATE mode of spc3d_sddmm for the sum of Z partial results
 *       (The PostComm phase; SpMM PostComm in "Building SpMM").
 *
 * Conventions for every call
 * --------------------------
 *  - "d_" pointers are device pointers on the plan's device; the caller owns
 *    all of them.  The library never allocates or frees device memory: a plan
 *    lives in a caller-provided workspace, and SpMM scratch space is a
 *    caller-provided buffer.
 *  - Every call returns an spc3d_status and never throws or aborts.
 *    spc3d_last_error() gives a thread-local text for the last failure.
 *  - Hot-path calls (gather, sddmm, spmm, scatter_reduce, permute, softmax)
 *    are asynchronous on `stream`; arguments are validated on the host before
 *    any launch.  Only spc3d_plan_create_coo synchronizes `stream`.
 *  - Dense row-major layouts: element (r, k) of a matrix with leading
 *    dimension ld is at offset r*ld + k.  Packed buffers have ld = kz.
 *  - Slot order: the plan stores the block's entries sorted by (local row,
 *    local column, caller index).  Values and SDDMM outputs passed to the hot
 *    calls are in this slot order; spc3d_permute_values converts from and to
 *    the caller's COO order.
 *  - Limits: nnz <= 2^31 - 65; each id range (hi - lo) in [1, 2^31 - 2];
 *    kz in [1, 1024] (kz not a multiple of the 16-byte vector width is limited
 *    to 256).
 *  - Distinct plans on distinct streams are independent.  Calls that share a
 *    plan only read it, so they may run concurrently unless they also share
 *    an output or an SpMM buffer.
 */
#ifndef SPC3D_H
#define SPC3D_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* The enum types below are int-sized.  C++ code sees them with int as fixed
 * underlying type, so any int a caller passes (say 7 for a dtype) is a value
 * the library's argument checks can reject, not an out-of-range enum. */
#ifdef __cplusplus
#define SPC3D_ENUM enum : int
#else
#define SPC3D_ENUM enum
#endif

typedef SPC3D_ENUM {
  SPC3D_OK = 0,
  SPC3D_ERR_INVALID_ARG = 1,  /* null pointer, bad size, misalignment, bad enum */
  SPC3D_ERR_OUT_OF_RANGE = 2, /* a global id outside [lo, hi) at plan creation */
  SPC3D_ERR_WORKSPACE = 3,    /* workspace or buffer smaller than required */
  SPC3D_ERR_UNSUPPORTED = 4,  /* valid request the library does not implement */
  SPC3D_ERR_HIP = 5,          /* a HIP runtime call failed */
  SPC3D_ERR_BAD_HANDLE = 6    /* not a live plan */
} spc3d_status;

typedef SPC3D_ENUM { SPC3D_F32 = 0, SPC3D_BF16 = 1 } spc3d_dtype;
typedef SPC3D_ENUM { SPC3D_ROWS = 0, SPC3D_COLS = 1 } spc3d_axis;

enum { SPC3D_OVERWRITE = 0, SPC3D_ACCUMULATE = 1 };  /* output modes */
enum { SPC3D_BUILD_CSC = 1u };                        /* plan flags */
enum { SPC3D_CALLER_TO_SLOT = 0, SPC3D_SLOT_TO_CALLER = 1,   /* spc3d_permute_values */
       SPC3D_SLOT_TO_COLUMN = 2, SPC3D_COLUMN_TO_SLOT = 3 };

/* Kernel variant for sddmm / spmm / sddmm_spmm: -1 lets the library choose
 * from kz, the operand type and the block's nnz;
 * otherwise (log2 of lanes per nonzero, 1..6) | (log2 of work-item slots / 64,
 * 0..4) << 4 | (SpMM gathers 16 rows per batch instead of 8, 0..1) << 8 |
 * SPC3D_VARIANT_WINDOW for the windowed SpMM family (each 64-slot window's
 * rows in flight together, row sums by a segmented scan; 2, 4 or 8 lanes,
 * not combined with the 16-row batches).  The SDDMM kernel ignores bits 8 and 9.  Every valid
 * variant computes the same result within the stated tolerance. */
#define SPC3D_VARIANT(lg_lanes, lg_items, wide) ((lg_lanes) | ((lg_items) << 4) | ((wide) << 8))
#define SPC3D_VARIANT_WINDOW 0x200

typedef struct spc3d_plan_s* spc3d_plan;

/* Device arrays of a plan (read-only views into its workspace).  R, C are the
 * numbers of non-empty rows / columns.  gmap_*: local -> global id (ascending);
 * lmap_*[g - lo]: global -> local id or -1; rowptr[R+1], colidx[nnz]: row-major
 * slots; perm[nnz]: slot -> caller index.  With SPC3D_BUILD_CSC also
 * colptr[C+1], rowidx_t[nnz] (local row of each column-major slot) and
 * slot_t[nnz] (row-major slot of each column-major slot); else NULL. */
typedef struct {
  const int64_t* gmap_r;
  const int64_t* gmap_c;
  const int32_t* lmap_r;
  const int32_t* lmap_c;
  const int32_t* rowptr;
  const int32_t* colidx;
  const int32_t* perm;
  const int32_t* colptr;
  const int32_t* rowidx_t;
  const int32_t* slot_t;
} spc3d_maps;

/* ------------------------------------------------------------------ setup */

/* Bytes of device workspace spc3d_plan_create_coo needs for a block with nnz
 * entries, row ids in [row_lo,row_hi) and column ids in [col_lo,col_hi). */
spc3d_status spc3d_plan_workspace_size(int64_t nnz, int64_t row_lo, int64_t row_hi,
                                       int64_t col_lo, int64_t col_hi, uint32_t flags,
                                       size_t* bytes);

/* Localize a block given in COO with global ids (paper: Section "Data
 * distribution"; the setup phase of Section "General structure").
 * d_row_gid[nnz], d_col_gid[nnz]: int64 global ids in caller order; repeated
 * (i,j) pairs are kept as separate entries.  Local ids are ranks of the
 * distinct ids in ascending order.  d_ws (256-byte aligned, ws_bytes from
 * spc3d_plan_workspace_size) must outlive the plan and is owned by it until
 * spc3d_plan_destroy.  Synchronizes `stream`.  Errors: INVALID_ARG,
 * WORKSPACE, OUT_OF_RANGE (any id outside its range; no plan is created). */
spc3d_status spc3d_plan_create_coo(spc3d_plan* out, int64_t nnz, const int64_t* d_row_gid,
                                   const int64_t* d_col_gid, int64_t row_lo, int64_t row_hi,
                                   int64_t col_lo, int64_t col_hi, uint32_t flags, void* d_ws,
                                   size_t ws_bytes, hipStream_t stream);

/* spc3d_plan_create_coo for a block given in CSR with global ids:
 * d_rowptr[row_hi - row_lo + 1] (int64) over every global row of the range
 * (rows without entries included), d_rowptr[0] = 0 and d_rowptr[last] =
 * nnz; d_col_gid[nnz] the int64 global column ids in row order.  The
 * "caller order" of values and of perm is the CSR entry order.  Same
 * workspace (spc3d_plan_workspace_size with this nnz), synchronization and
 * errors as spc3d_plan_create_coo, plus INVALID_ARG for a row pointer that
 * does not start at 0, decreases, or does not end at nnz. */
spc3d_status spc3d_plan_create_csr(spc3d_plan* out, int64_t nnz, const int64_t* d_rowptr,
                                   const int64_t* d_col_gid, int64_t row_lo, int64_t row_hi,
                                   int64_t col_lo, int64_t col_hi, uint32_t flags, void* d_ws,
                                   size_t ws_bytes, hipStream_t stream);

/* spc3d_plan_create_coo with the owner-grouped local order of Method 2
 * (SpC-SB / SpC-RB) of Section "Sparse communication model": local data
 * stored as the concatenation of the data units exchanged with each peer, so
 * that each message is sent or received in place.  d_group_r (int32, one key
 * per id of [row_lo, row_hi), or NULL for ascending ids) gives every row id a
 * group in [0, ngroups_r), 1 <= ngroups_r <= 4096 (for example 0 for the rows
 * this processor owns and 1 + the owner's rank among its peers for the
 * others); local rows are then the distinct ids ordered by (group, global
 * id), and the CSR, the maps and every packed buffer follow that order.
 * Likewise d_group_c / ngroups_c for columns.  Keys of ids the block does not
 * use are ignored; a used id with a key outside [0, ngroups) gives
 * INVALID_ARG and no plan.  Same workspace, synchronization and errors as
 * spc3d_plan_create_coo. */
spc3d_status spc3d_plan_create_coo_grouped(spc3d_plan* out, int64_t nnz,
                                           const int64_t* d_row_gid, const int64_t* d_col_gid,
                                           int64_t row_lo, int64_t row_hi, int64_t col_lo,
                                           int64_t col_hi, const int32_t* d_group_r,
                                           int32_t ngroups_r, const int32_t* d_group_c,
                                           int32_t ngroups_c, uint32_t flags, void* d_ws,
                                           size_t ws_bytes, hipStream_t stream);

/* Device view of a grouped axis: *d_offsets points at ngroups + 1 int32 in
 * the plan's workspace, offsets[q] = first local id of group q and
 * offsets[ngroups] = R (or C): group q occupies local ids [offsets[q],
 * offsets[q+1]), i.e. rows [offsets[q], offsets[q+1]) of a packed buffer.
 * INVALID_ARG if the axis was built without groups. */
spc3d_status spc3d_plan_group_offsets(spc3d_plan plan, spc3d_axis axis,
                                      const int32_t** d_offsets, int32_t* ngroups);

/* Sizes of a plan: non-empty rows R, non-empty columns C, entries nnz. */
spc3d_status spc3d_plan_query(spc3d_plan plan, int64_t* R, int64_t* C, int64_t* nnz);

/* Device views of a plan's maps and index arrays (see spc3d_maps). */
spc3d_status spc3d_plan_maps(spc3d_plan plan, spc3d_maps* maps);

/* Release the host object; the workspace may be reused afterwards. */
spc3d_status spc3d_plan_destroy(spc3d_plan plan);

/* Checks, on the device, every local id of the plan that the gather,
 * scatter-reduce, permute and compute kernels turn into an address (the
 * localization's output, Section "The setup phase"): rowptr [R+1] runs from
 * 0 to nnz and strictly increases; colidx[s] lies in [0, C); the head bitmap
 * marks exactly the slots rowptr[r] and nothing past nnz; tile_row[t] is the
 * row of slot 64t; perm[s] lies in [0, nnz); gmap_r / gmap_c lie in the
 * block's row / column range and ascend (unless owner-grouped); and the same
 * for the column-major arrays of a plan built with SPC3D_BUILD_CSC.  Reads
 * only the plan's arrays, never through their values, so a damaged plan
 * cannot make it fault.  Synchronizes `stream` (not for use under graph
 * capture); the check uses one device word per GPU held by the library, so
 * checks that overlap on one GPU race.  Returns OK, or OUT_OF_RANGE with
 * spc3d_last_error() naming the first violated invariant and its index. */
spc3d_status spc3d_plan_check(spc3d_plan plan, hipStream_t stream);

/* 1 when the environment variable SPC3D_DEBUG_BOUNDS is set to anything but
 * "0" (read once per process): every call that launches kernels over a plan
 * then runs spc3d_plan_check on it first, on its stream, and returns that
 * check's error instead of launching.  0 otherwise (no checking, no cost). */
int spc3d_debug_bounds(void);

/* -------------------------------------------------------------- hot path */

/* PreComm, local side: SpC-BB packing of data units (paper: Section "Sparse
 * communication model", Method 1).  axis ROWS packs n = R rows, COLS n = C:
 *   d_packed[l*kz + k] = d_src[(gmap[l] - lo)*ld_src + k0 + k],  l < n, k < kz.
 * d_src rows are indexed relative to the axis' lo.  src_t F32 -> packed_t F32
 * (bit copy) or BF16 (round to nearest even; NaN stays NaN with its sign);
 * src_t BF16 -> packed_t BF16 (bit copy).  Requires 0 <= k0, k0 + kz <= ld_src. */
spc3d_status spc3d_gather(spc3d_plan plan, spc3d_axis axis, const void* d_src,
                          spc3d_dtype src_t, int64_t ld_src, int32_t k0, int32_t kz,
                          void* d_packed, spc3d_dtype packed_t, hipStream_t stream);

/* SDDMM, Eq. (1), over the localized block: for every slot p with local row
 * i and local column j,
 *   d_out[p] (=|+=) s_p * sum_{k<kz} A[i*kz + k] * B[j*kz + k]
 * d_vals[nnz] in slot order (NULL: s == 1, pattern-only sampling); d_A
 * [R x kz] and d_B [C x kz] packed, of type ab_t (F32, or BF16 with FP32
 * accumulation); d_out[nnz] FP32 in slot order.  mode OVERWRITE or
 * ACCUMULATE (adds this K-slice's partial to d_out: the Z-partial sum of the
 * SDDMM PostComm).  d_out may not alias the inputs. */
spc3d_status spc3d_sddmm(spc3d_plan plan, const float* d_vals, const void* d_A, const void* d_B,
                         spc3d_dtype ab_t, int32_t kz, float* d_out, int mode, int variant,
                         hipStream_t stream);

/* Bytes of scratch spc3d_spmm and spc3d_sddmm_spmm need for (transpose, kz,
 * variant): enough for either operand type, aligned or not, fused or not.
 * Errors: INVALID_ARG or UNSUPPORTED when no shape of `variant` fits kz. */
spc3d_status spc3d_spmm_buffer_size(spc3d_plan plan, int transpose, int32_t kz, int variant,
                                    size_t* bytes);

/* SpMM, Eq. (2), over the localized block:
 *   transpose = 0:  Y[i*kz + k] (=|+=) sum_{p in row i} s_p * X[j(p)*kz + k],
 *                   X [C x kz], Y [R x kz];
 *   transpose = 1:  Y[j*kz + k] (=|+=) sum_{p in column j} s_p * X[i(p)*kz + k],
 *                   X [R x kz], Y [C x kz]  (needs a plan built with
 *                   SPC3D_BUILD_CSC; used by the backward of SDDMM / SpMM);
 *   transpose = 2:  as 1, with d_vals in column-major order (as
 *                   spc3d_permute_values SLOT_TO_COLUMN gives), read as one
 *                   stream instead of through the slot map; same results.
 * d_vals[nnz] FP32 in slot order (NULL: s == 1) unless transpose = 2.  X of type x_t (F32 or BF16),
 * accumulation and Y in FP32.  Long rows are split across wavefronts and their
 * partial sums combined in a fixed order, so results are deterministic.
 * d_buf (256-byte aligned) holds at least spc3d_spmm_buffer_size bytes.
 * Y may not alias X. */
spc3d_status spc3d_spmm(spc3d_plan plan, int transpose, const float* d_vals, const void* d_X,
                        spc3d_dtype x_t, int32_t kz, float* d_Y, int mode, int variant,
                        void* d_buf, size_t buf_bytes, hipStream_t stream);

/* SDDMM and SpMM of the same block in one pass over its slots (the pattern
 * the paper's comparison runs: SDDMM followed by SpMM with the same sparse
 * matrix and the same B rows; Section "Experimental Evaluation").  Computes
 *   d_out[p] (=|+=) s_p * <A[i(p)], B[j(p)]>          (as spc3d_sddmm)
 *   d_Y[i]   (=|+=) sum_{p in row i} s_p * B[j(p)]    (as spc3d_spmm, transpose 0)
 * reading each entry's packed B row once for both.  Arguments as for
 * spc3d_sddmm and spc3d_spmm; d_buf holds spc3d_spmm_buffer_size(plan, 0, kz,
 * variant) bytes.  Neither output may alias an input. */
spc3d_status spc3d_sddmm_spmm(spc3d_plan plan, const float* d_vals, const void* d_A,
                              const void* d_B, spc3d_dtype ab_t, int32_t kz, float* d_out,
                              float* d_Y, int mode, int variant, void* d_buf, size_t buf_bytes,
                              hipStream_t stream);

/* The fused pass with the SpMM PostComm folded in: SDDMM values as
 * spc3d_sddmm_spmm computes them, and each local row's SpMM sum added straight
 * into the owner's slab instead of a packed Y (Section "Building SpMM with
 * SpComm3D": partial rows reduced at their owner; Method 1 unpacking):
 *   d_out[p] (=|+=) s_p * <A[i(p)], B[j(p)]>            (out_mode)
 *   d_dst[(gmap_r[i] - row_lo)*ld_dst + k0 + k] += sum_{p in row i} s_p * B[j(p)*kz + k]
 * for every local row i and k < kz.  Each row sum is complete (summed in the
 * same order as spc3d_sddmm_spmm) before its single addition, so d_dst ends
 * bit for bit as after spc3d_sddmm_spmm (OVERWRITE) followed by
 * spc3d_scatter_reduce(ROWS); rows the block does not touch are unchanged.
 * Requires 0 <= k0, k0 + kz <= ld_dst; d_dst may not alias an input.  d_buf
 * holds spc3d_spmm_buffer_size(plan, 0, kz, variant) bytes. */
spc3d_status spc3d_sddmm_spmm_scatter(spc3d_plan plan, const float* d_vals, const void* d_A,
                                      const void* d_B, spc3d_dtype ab_t, int32_t kz, float* d_out,
                                      int out_mode, float* d_dst, int64_t ld_dst, int32_t k0,
                                      int variant, void* d_buf, size_t buf_bytes,
                                      hipStream_t stream);

/* Bytes of the library's static scratch array (one per GPU) that
 * spc3d_sddmm_spmm_static uses in place of a caller buffer. */
#define SPC3D_STATIC_SCRATCH_BYTES (16u << 20)

/* spc3d_sddmm_spmm for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same computation and results, with the SpMM carries kept in a device
 * array of SPC3D_STATIC_SCRATCH_BYTES that the library holds on each GPU it
 * runs on until the process ends, so no scratch argument is taken and nothing
 * is allocated or freed.  The caller still owns the inputs and outputs.
 * Every call on one GPU shares that GPU's array and leaves its contents
 * behind: calls that overlap on one GPU (on different streams, or from
 * different threads) race and must be ordered by the caller.  A call whose
 * carries need more than SPC3D_STATIC_SCRATCH_BYTES (2 * kz * 4 bytes per
 * work item; e.g. 16 MiB covers 4M entries at kz = 128 in the default shape)
 * returns SPC3D_ERR_WORKSPACE before any launch.  Other errors as for
 * spc3d_sddmm_spmm. */
spc3d_status spc3d_sddmm_spmm_static(spc3d_plan plan, const float* d_vals, const void* d_A,
                                     const void* d_B, spc3d_dtype ab_t, int32_t kz, float* d_out,
                                     float* d_Y, int mode, int variant, hipStream_t stream);

/* PostComm, local side: SpC-BB unpacking with reduction at the owner (paper:
 * "Building SpMM with SpComm3D", partial A rows sent to their owners):
 *   d_dst[(gmap[l] - lo)*ld_dst + k0 + k] += d_packed[l*kz + k]   (IEEE FP32)
 * for l < n (R for ROWS, C for COLS), k < kz.  Rows of d_dst that the block
 * does not touch are left unchanged.  Requires 0 <= k0, k0 + kz <= ld_dst. */
spc3d_status spc3d_scatter_reduce(spc3d_plan plan, spc3d_axis axis, const float* d_packed,
                                  int32_t kz, float* d_dst, int64_t ld_dst, int32_t k0,
                                  hipStream_t stream);

/* Move per-entry FP32 values between caller (COO) order and slot order:
 * CALLER_TO_SLOT: out[p] = in[perm[p]];  SLOT_TO_CALLER: out[perm[p]] = in[p];
 * or between slot order and the column-major order of a plan built with
 * SPC3D_BUILD_CSC: SLOT_TO_COLUMN: out[t] = in[slot_t[t]];
 * COLUMN_TO_SLOT: out[slot_t[t]] = in[t].  in and out must not alias. */
spc3d_status spc3d_permute_values(spc3d_plan plan, int direction, const float* d_in,
                                  float* d_out, hipStream_t stream);

/* -------------------------------------------------- graph attention (ext.) */

/* Bytes of scratch spc3d_row_softmax / spc3d_row_softmax_bwd need. */
spc3d_status spc3d_row_softmax_buffer_size(spc3d_plan plan, size_t* bytes);

/* Row-wise softmax over each row's stored entries (slot order):
 *   alpha[p] = exp(e[p] - max_row) / sum_{q in row} exp(e[q] - max_row).
 * Used between the SDDMM scores and the SpMM aggregation of a graph-attention
 * layer.  d_e and d_alpha hold nnz FP32 values and may alias; d_buf
 * (256-byte aligned) holds at least spc3d_row_softmax_buffer_size bytes. */
spc3d_status spc3d_row_softmax(spc3d_plan plan, const float* d_e, float* d_alpha, void* d_buf,
                               size_t buf_bytes, hipStream_t stream);

/* Backward of spc3d_row_softmax:
 *   de[p] = alpha[p] * (dalpha[p] - sum_{q in row} alpha[q] * dalpha[q]).
 * d_de may alias d_dalpha; d_buf as for spc3d_row_softmax. */
spc3d_status spc3d_row_softmax_bwd(spc3d_plan plan, const float* d_alpha, const float* d_dalpha,
                                   float* d_de, void* d_buf, size_t buf_bytes,
                                   hipStream_t stream);

/* alpha[p] = exp(e[p] - stats[2r]) / stats[2r+1] for every entry p of local
 * row r: the softmax weights rebuilt from scores and the per-row (max, sum of
 * exp(e - max)) that spc3d_attention_fwd stores.  d_stats holds 2R floats
 * (8-byte aligned); d_e and d_alpha hold nnz values and may alias. */
spc3d_status spc3d_row_softmax_apply(spc3d_plan plan, const float* d_e, const float* d_stats,
                                     float* d_alpha, hipStream_t stream);

/* Bytes of scratch spc3d_attention_fwd needs for (kz, dtype, variant). */
spc3d_status spc3d_attention_fwd_buffer_size(spc3d_plan plan, int32_t kz, spc3d_dtype t,
                                             int variant, size_t* bytes);

/* Fused masked attention forward over the block's pattern (the SDDMM ->
 * softmax -> SpMM chain of a graph-attention layer in one pass; an extension
 * built on Eq. (1) and Eq. (2)):
 *   e_p = sum_k Q[r*kz + k] * K[c*kz + k]               (entry p = (r, c))
 *   out[r*kz + k] = sum_{p in row r} exp(e_p - m_r) / s_r * V[c*kz + k]
 * with m_r = max of row r's scores and s_r = sum_{p in row r} exp(e_p - m_r);
 * d_stats (2R floats, 8-byte aligned, may be NULL) receives (m_r, s_r).
 * Q is [R x kz], K and V are [C x kz], packed row-major, 16-byte aligned, of
 * type t (FP32 or bfloat16); out is [R x kz] FP32.  Scores never reach
 * memory; each row's partial (max, sum, weighted sum) triples are merged by
 * rescaling to the larger maximum in an order fixed by the pattern, so the
 * result is deterministic.  kz*sizeof(t) must be 64, 128, 256 or 512 bytes
 * (FP32 kz 16, 32, 64, 128; bfloat16 kz 32, 64, 128, 256), else
 * SPC3D_ERR_UNSUPPORTED (sddmm, row_softmax and spmm compute the same).
 * Scores of -inf: a row whose scores are all -inf gives the mean of its V
 * rows rather than NaN.
 * variant: -1, or lg2(lanes per entry) (2..4) | lg2(slots per lane group)
 * << 4 (4..6).  d_buf (256-byte aligned) holds at least
 * spc3d_attention_fwd_buffer_size bytes.  Asynchronous on stream. */
spc3d_status spc3d_attention_fwd(spc3d_plan plan, const void* d_Q, const void* d_K,
                                 const void* d_V, spc3d_dtype t, int32_t kz, float* d_out,
                                 float* d_stats, int variant, void* d_buf, size_t buf_bytes,
                                 hipStream_t stream);

/* Per-entry product out[p] = a[p] * b[p] for the nnz entries of a plan (slot
 * order).  The backward of SDDMM scales the upstream gradient by the sampling
 * values with it: d(s_p <a_i,b_j>)/d a_i = s_p b_j.  Any of the arrays may
 * alias. */
spc3d_status spc3d_mul_values(spc3d_plan plan, const float* d_a, const float* d_b, float* d_out,
                              hipStream_t stream);

/* ------------------------------- communication accounting (Dist3D) */

/* Bytes of device workspace spc3d_lambda_owners needs for ids [lo, hi). */
spc3d_status spc3d_lambda_owners_workspace_size(int64_t lo, int64_t hi, size_t* bytes);

/* lambda counts and Algorithm 1's owner choice for one block row (or column)
 * of a Dist3D grid (Section "Sparsity-aware Communication Analysis of 3D
 * SDDMM"; Algorithm 1, "Parallel lambda-aware random distribution").  Part p
 * (0 <= p < nparts <= 64) uses the h_counts[p] distinct global ids of the
 * device array h_gmaps[p] (e.g. a plan's gmap_r), all in [lo, hi).  For every
 * id i in [lo, hi), with j = i - lo:
 *   d_lambda[j] = number of parts that use i;
 *   d_owner[j]  = the part of rank floor(d_rand[j] * lambda / 2^64) among
 *                 them in ascending order (rank 0 when d_rand is NULL), or -1
 *                 when no part uses i;
 *   d_owned[p]  = number of ids part p owns;
 *   d_comm[p*nparts + q] = number of ids part p uses and part q != p owns
 *                 (the rows p receives from q), 0 on the diagonal.
 * Integer results, independent of scheduling.  d_rand holds hi - lo 64-bit
 * random numbers (the caller's seeded draws).  h_gmaps and h_counts are host
 * arrays of nparts entries.  A setup-time call: it synchronizes the stream
 * and returns SPC3D_ERR_OUT_OF_RANGE when a part holds an id outside
 * [lo, hi) (such ids are skipped). */
spc3d_status spc3d_lambda_owners(int32_t nparts, const int64_t* const* h_gmaps,
                                 const int64_t* h_counts, int64_t lo, int64_t hi,
                                 const uint64_t* d_rand, int32_t* d_lambda, int32_t* d_owner,
                                 int64_t* d_owned, int64_t* d_comm, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream);

/* ------------------------------------- learned variant selector (ext.) */

/* Operations a variant is chosen for: spc3d_sddmm, spc3d_spmm (transpose 0)
 * and spc3d_sddmm_spmm. */
enum { SPC3D_OP_SDDMM = 0, SPC3D_OP_SPMM = 1, SPC3D_OP_SDDMM_SPMM = 2 };

/* Host-only: SPC3D_OK when `variant` (or -1, the default shape) can run
 * operation `op` on 16-byte aligned packed operands of type ab_t with this
 * kz; SPC3D_ERR_UNSUPPORTED when the shape does not fit kz (too few lanes, or
 * too few slots per lane group for SpMM); SPC3D_ERR_INVALID_ARG for a
 * malformed variant, op, dtype or kz.  Launches nothing. */
spc3d_status spc3d_variant_check(int op, int32_t kz, spc3d_dtype ab_t, int variant);

/* Number of features spc3d_plan_features writes, and the device scratch
 * (8-byte aligned) it needs. */
#define SPC3D_NFEAT 23
#define SPC3D_FEATURES_BUFFER_BYTES 256

/* Sparsity features of one orientation of a plan (transpose 0: rows of the
 * CSR view; 1: columns, needs SPC3D_BUILD_CSC), for an operation on packed
 * operands of type ab_t with K-slice kz.  d_out[SPC3D_NFEAT] (FP32, device):
 *   [0,16)  fraction of the nnz entries that lie in rows whose length is in
 *           [2^b, 2^(b+1)) (b = 15 also takes every longer row)
 *   16 log2(longest row)/16   17 log2(rows)/16   18 log2(columns)/16
 *   19 log2(nnz)/24           20 log2(nnz/rows)/8
 *   21 log2(kz)/8             22 1 for BF16 operands, 0 for FP32
 * (log2 of a value below 1 is taken as 0).  Integer counts are exact; each
 * fraction is the FP64 quotient rounded to FP32.  d_buf holds
 * SPC3D_FEATURES_BUFFER_BYTES bytes of scratch. */
spc3d_status spc3d_plan_features(spc3d_plan plan, int transpose, int32_t kz, spc3d_dtype ab_t,
                                 float* d_out, void* d_buf, size_t buf_bytes, hipStream_t stream);

/* Dense layer of the selector's multilayer perceptron (FP32, device arrays,
 * row-major): Y[n x fout] = act(X[n x fin] W[fout x fin]^T + b[fout]), act the
 * identity (relu = 0) or max(0, .) (relu = 1).  d_b may be NULL (no bias).
 * Limits: 1 <= fin, fout <= 1024, 0 <= n <= 2^20, n * max(fin, fout) <=
 * 65535 * 256.  Y may not alias X. */
spc3d_status spc3d_mlp_linear_fwd(int n, int fin, int fout, const float* d_X, const float* d_W,
                                  const float* d_b, float* d_Y, int relu, hipStream_t stream);

/* Bytes of scratch spc3d_mlp_linear_bwd needs for (n, fin, fout). */
spc3d_status spc3d_mlp_linear_bwd_buffer_size(int n, int fin, int fout, size_t* bytes);

/* Backward of spc3d_mlp_linear_fwd given the upstream gradient dY [n x fout]:
 * with G = dY masked by Y > 0 when relu = 1 (the derivative at 0 taken as 0),
 *   dX = G W (skipped when d_dX is NULL),  dW = G^T X,  db = column sums of G
 * (skipped when d_db is NULL).  d_Y is the forward output (read only when
 * relu = 1).  Reductions over n run in a fixed order (deterministic).  d_buf
 * (4-byte aligned) holds spc3d_mlp_linear_bwd_buffer_size bytes. */
spc3d_status spc3d_mlp_linear_bwd(int n, int fin, int fout, const float* d_X, const float* d_W,
                                  const float* d_Y, const float* d_dY, int relu, float* d_dX,
                                  float* d_dW, float* d_db, void* d_buf, size_t buf_bytes,
                                  hipStream_t stream);

/* Masked mean squared error over n entries: with c = sum mask (1 if 0),
 *   loss = sum mask (P - T)^2 / c,   dP = 2 mask (P - T) / c.
 * d_loss (one float) may be NULL.  One workgroup; fixed summation order. */
spc3d_status spc3d_mlp_mse(int64_t n, const float* d_P, const float* d_T, const float* d_mask,
                           float* d_dP, float* d_loss, hipStream_t stream);

/* One Adam step (Kingma and Ba, 2015) at step count `step` >= 1 on n
 * parameters w with gradient g and moment estimates m, v (updated in place):
 *   m = b1 m + (1-b1) g;  v = b2 v + (1-b2) g^2;
 *   w -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
spc3d_status spc3d_mlp_adam(int64_t n, float* d_w, const float* d_g, float* d_m, float* d_v,
                            float lr, float beta1, float beta2, float eps, int step,
                            hipStream_t stream);

/* idx[r] = the least-P column o among those with mask[r*m + o] != 0 (the
 * first on ties), -1 when a row has none; P and mask [n x m] FP32.  With
 * 0 <= pref < m, idx[r] = pref instead when pref is allowed in row r and
 * P[r*m + pref] <= P[r*m + o] + margin (an FP32 sum): a preferred column
 * (the selector's default shape) kept unless another is predicted better by
 * more than margin.  pref = -1 for none; margin finite and >= 0. */
spc3d_status spc3d_mlp_masked_argmin(int n, int m, const float* d_P, const float* d_mask,
                                     int32_t pref, float margin, int32_t* d_idx,
                                     hipStream_t stream);

/* ----------------------------------------------------------- diagnostics */

const char* spc3d_status_string(spc3d_status status);
const char* spc3d_last_error(void);
/* Library version as major*10000 + minor*100 + patch. */
int spc3d_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPC3D_H */
