// Compute phase: SDDMM, Eq. (1), and SpMM, Eq. (2), over a localized block
// with a K-slice of width kz (paper: Section "Building 3D SDDMM and SpMM
// Algorithms", The Compute phase — each of the Z instances forms the inner
// products over K/Z columns; "Building SpMM" for the row-wise SpMM).
//
// Work decomposition (both kernels).  The block's slots are cut into work
// items of W consecutive slots (W a multiple of 64), one item per wavefront,
// regardless of row boundaries, so power-law hub rows cannot serialize a
// wavefront.  A wavefront is split into G = 64 / L groups of L lanes; a group
// owns one nonzero at a time and each lane of it holds NCH vectors of VEC
// elements of the kz-wide dense row (16-byte loads: 4 FP32 or 8 bfloat16).
// Rows are recovered from a 64-bit head bitmap per 64 slots plus the row of
// the tile's first slot (a popcount), so no per-slot row array is read.
//
// SDDMM: in each 64-slot window, group g computes the dots of slots
// g*L .. g*L+L-1 one after another (lane-parallel FMAs, then an xor-butterfly
// over the L lanes); lane i ends up holding slot i's dot and the window's 64
// outputs are written with one coalesced store.
//
// SpMM: group g walks a contiguous run of S = W / G slots, accumulating
// s_p * X[col] in registers; a row that starts and ends inside the run is
// written directly.  Rows cut by run boundaries leave partial sums in LDS
// (the first row of a run) or registers (the last); after one barrier the
// group that started such a row adds the following runs' partials in run
// order.  Rows cut by item boundaries leave per-item carries that a small
// second kernel adds in item order (blocked, then a butterfly across groups).
// The summation order depends only on the structure, so results are
// deterministic, and every FP32 sum has depth O(S + G + W-items / 16), which
// keeps the rounding error far inside 1e-5 of the magnitude sum even for rows
// with 10^5 entries.
#pragma once

#include "internal.h"
#include "vec.h"

namespace spc3d {

enum { kLeadNone = 0, kLeadEnds = 1, kLeadThrough = 2 };

// Streaming accesses (indices and values read once, outputs written once)
// carry the nontemporal hint so that they do not displace the dense rows
// that later entries gather again from L2.
#ifndef SPC3D_STREAM_HINTS
#define SPC3D_STREAM_HINTS 1
#endif
template <typename T>
__device__ inline T ld_stream(const T* p) {
#if SPC3D_STREAM_HINTS
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}
template <typename T>
__device__ inline void st_stream(T* p, T v) {
#if SPC3D_STREAM_HINTS
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Row of slot s from the head bitmap.
__device__ inline int row_of(const uint64_t* __restrict__ head, const int32_t* __restrict__ tile_row,
                             int64_t s) {
  return tile_row[s >> 6] + __popcll(head[s >> 6] & lanemask_le((int)(s & 63)) & ~1ull);
}

__device__ inline bool is_head(const uint64_t* __restrict__ head, int64_t s) {
  return (head[s >> 6] >> (s & 63)) & 1ull;
}

// Sum of v over the L lanes of a group (a butterfly: DPP within 16-lane
// rows, cross-lane permutes beyond).  Every lane of the group gets the sum.
template <int LPN>
__device__ inline float group_sum(float v) {
  if constexpr (LPN >= 2)
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
  if constexpr (LPN >= 4)
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
  if constexpr (LPN >= 8)
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x141, 0xF, 0xF, false));
  if constexpr (LPN >= 16)
    v += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x140, 0xF, 0xF, false));
  if constexpr (LPN >= 32) v += __shfl_xor(v, 16);
  if constexpr (LPN >= 64) v += __shfl_xor(v, 32);
  return v;
}

// Loads this lane's NCH vectors of a kz-wide row.  Vectors past the row end
// (lanes left over when kz/VEC is not a multiple of L) re-read the last
// vector so that no load is predicated; callers ignore them.
template <typename T, int VEC, int LPN, int NCH>
__device__ inline void load_row(const T* __restrict__ row, int q, int nvec, float (&x)[NCH][VEC]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    int vi = q + ch * LPN;
    vi = vi < nvec ? vi : nvec - 1;
    VecLoad<T, VEC>::load(row + vi * VEC, x[ch]);
  }
}

template <int VEC, int LPN, int NCH>
__device__ inline float lane_dot(const float (&a)[NCH][VEC], const float (&b)[NCH][VEC], int q,
                                 int nvec) {
  float acc = 0.f;
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const bool on = q + ch * LPN < nvec;
#pragma unroll
    for (int t = 0; t < VEC; ++t) {
      const float f = fmaf(a[ch][t], b[ch][t], acc);
      acc = on ? f : acc;
    }
  }
  return acc;
}

// ------------------------------------------------------------------ SDDMM

template <typename T, int VEC, int LPN, int NCH>
__global__ __launch_bounds__(256) void k_sddmm(int64_t nnz, int64_t nitems, int64_t nblocks,
                                               int wslots, const int32_t* __restrict__ colidx,
                                               const uint64_t* __restrict__ head,
                                               const int32_t* __restrict__ tile_row,
                                               const float* __restrict__ vals,
                                               const T* __restrict__ A, const T* __restrict__ B,
                                               int kz, float* __restrict__ out, int accumulate) {
  // JB nonzeros per group have their rows in flight together (2*JB*NCH*VEC
  // registers of loads).
  constexpr int JB0 = 64 / (2 * NCH * VEC);
  constexpr int JB = JB0 < 1 ? 1 : (JB0 > LPN ? LPN : JB0);
  const int lane = threadIdx.x & 63;
  const int g = lane / LPN, q = lane % LPN;
  const int64_t item = xcd_block(nblocks) * 4 + (threadIdx.x >> 6);
  if (item >= nitems) return;   // uniform per wavefront; no barriers below
  const int nvec = kz / VEC;
  const int64_t b = item * wslots;
  const int64_t e = (b + wslots < nnz) ? b + wslots : nnz;
  for (int64_t win = b; win < e; win += 64) {
    const int64_t s = win + lane;
    const bool valid = s < e;
    const int col = valid ? ld_stream(colidx + s) : 0;
    const float v = vals ? (valid ? ld_stream(vals + s) : 0.f) : 1.f;
    // lanes past the end repeat the last valid row (no head bits there)
    const int row = tile_row[win >> 6] + __popcll(head[win >> 6] & lanemask_le(lane) & ~1ull);
    float res = 0.f;
#pragma unroll
    for (int j0 = 0; j0 < LPN; j0 += JB) {
      float a[JB][NCH][VEC], bb[JB][NCH][VEC];
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const int src = g * LPN + j0 + jj;
        const int c = __shfl(col, src);
        const int r = __shfl(row, src);
        load_row<T, VEC, LPN, NCH>(A + (int64_t)r * kz, q, nvec, a[jj]);
        load_row<T, VEC, LPN, NCH>(B + (int64_t)c * kz, q, nvec, bb[jj]);
      }
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const float d = group_sum<LPN>(lane_dot<VEC, LPN, NCH>(a[jj], bb[jj], q, nvec));
        if (q == j0 + jj) res = d;
      }
    }
    if (valid) {
      const float o = v * res;
      st_stream(out + s, accumulate ? ld_stream(out + s) + o : o);
    }
  }
}

// ------------------------------------------------------------------- SpMM

// Stores (or, with accumulate, adds) this lane's part of a finished row sum
// at yr, the first element of the destination row.
template <int VEC, int NCH>
__device__ inline void store_row_at(float* __restrict__ yr, int nvec, int q, int lpn,
                                    const float (&acc)[NCH][VEC], int accumulate) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int vi = q + ch * lpn;
    if (vi < nvec) {
      float* y = yr + vi * VEC;
      if constexpr (VEC % 4 == 0) {
#pragma unroll
        for (int t = 0; t < VEC; t += 4) {
          f32x4 o = {acc[ch][t], acc[ch][t + 1], acc[ch][t + 2], acc[ch][t + 3]};
          if (accumulate) o = ld_stream(reinterpret_cast<const f32x4*>(y + t)) + o;
          st_stream(reinterpret_cast<f32x4*>(y + t), o);
        }
      } else {
#pragma unroll
        for (int t = 0; t < VEC; ++t) y[t] = accumulate ? y[t] + acc[ch][t] : acc[ch][t];
      }
    }
  }
}

template <int VEC, int NCH>
__device__ inline void store_row(float* __restrict__ Y, int64_t row, int kz, int nvec, int q,
                                 int lpn, const float (&acc)[NCH][VEC], int accumulate) {
  store_row_at<VEC, NCH>(Y + row * kz, nvec, q, lpn, acc, accumulate);
}

// Where the SpMM kernels put a finished row r: at base + r * ld (the packed
// Y_loc, ld = kz), or, with map set, added into the owner's slab at
// base + (map[r] - lo) * ld, which is the PostComm scatter-reduce of Y_loc
// done as each row completes (base then points at column k0 of row lo).
// Every row is finished, and so stored, exactly once.
struct YOut {
  float* base;
  const int64_t* map;
  int64_t lo;
  int64_t ld;
  int64_t n;   // entries of map (the local rows)
};

// Bits of the kernels' accumulate argument: add SpMM rows into the
// destination; add SDDMM values into out (the fused pass).
enum { kAccY = 1, kAccOut = 2 };

template <int VEC, int NCH>
__device__ inline void store_row(const YOut& Y, int64_t row, int /*kz*/, int nvec, int q, int lpn,
                                 const float (&acc)[NCH][VEC], int accumulate) {
  const int64_t r = Y.map ? Y.map[row] - Y.lo : row;
  store_row_at<VEC, NCH>(Y.base + r * Y.ld, nvec, q, lpn, acc, accumulate & kAccY);
}

// This lane's part of a destination row (VEC a multiple of 4), loaded ahead of
// the addition that completes the row.
template <int VEC, int NCH>
__device__ inline void load_dst(const float* __restrict__ yr, int nvec, int q, int lpn,
                                float (&pre)[NCH][VEC]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int vi = q + ch * lpn;
    if (vi < nvec) {
#pragma unroll
      for (int t = 0; t < VEC; t += 4) {
        const f32x4 v = ld_stream(reinterpret_cast<const f32x4*>(yr + vi * VEC + t));
        pre[ch][t] = v.x; pre[ch][t + 1] = v.y; pre[ch][t + 2] = v.z; pre[ch][t + 3] = v.w;
      }
    }
  }
}

// yr = pre + acc, the finished row added to the destination values loaded
// when the row started (the same FP32 addition as a read-modify-write).
template <int VEC, int NCH>
__device__ inline void store_pre(float* __restrict__ yr, int nvec, int q, int lpn,
                                 const float (&pre)[NCH][VEC], const float (&acc)[NCH][VEC]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int vi = q + ch * lpn;
    if (vi < nvec) {
#pragma unroll
      for (int t = 0; t < VEC; t += 4) {
        const f32x4 o = {pre[ch][t] + acc[ch][t], pre[ch][t + 1] + acc[ch][t + 1],
                         pre[ch][t + 2] + acc[ch][t + 2], pre[ch][t + 3] + acc[ch][t + 3]};
        st_stream(reinterpret_cast<f32x4*>(yr + vi * VEC + t), o);
      }
    }
  }
}

template <int VEC, int NCH>
__device__ inline void store_vec(float* __restrict__ dst, int nvec, int q, int lpn,
                                 const float (&acc)[NCH][VEC]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int vi = q + ch * lpn;
    if (vi < nvec) {
#pragma unroll
      for (int t = 0; t < VEC; ++t) dst[vi * VEC + t] = acc[ch][t];
    }
  }
}

template <int VEC, int NCH>
__device__ inline void add_vec(const float* __restrict__ src, int nvec, int q, int lpn,
                               float (&acc)[NCH][VEC]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int vi = q + ch * lpn;
    if (vi < nvec) {
#pragma unroll
      for (int t = 0; t < VEC; ++t) acc[ch][t] += src[vi * VEC + t];
    }
  }
}

template <int VEC, int NCH>
__device__ inline void zero(float (&acc)[NCH][VEC]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
    for (int t = 0; t < VEC; ++t) acc[ch][t] = 0.f;
}

// LDS bytes one wavefront of k_spmm uses (fused: plus the SDDMM outputs).
// Staged per-slot arrays hold one pad word per run of S = W/G slots, so the
// G groups reading slot u of their runs hit different LDS banks.
// The item's head words and tile rows (12 bytes per 64 slots) are staged too,
// so no batch waits on a global load before it can address its rows.
__host__ __device__ inline size_t spmm_wave_lds(int wslots, int lpn, int nch, int vec, bool fused) {
  const int G = 64 / lpn;
  const size_t P = (size_t)wslots + G;
  const size_t bytes = P * (fused ? 12 : 8) + (size_t)G * lpn * nch * vec * 4 + (size_t)G * 4 +
                       (size_t)(wslots / 64) * 12;
  return (bytes + 15) & ~(size_t)15;   // keeps every wave's 8-byte head words aligned
}

// One batch of UB consecutive slots of a group: their columns, values, head
// bits and the rows they gather (and, fused, the A rows of their own rows).
template <typename T, int VEC, int LPN, int NCH, int UB, bool FUSED>
struct Batch {
  float x[UB][NCH][VEC];
  float a[FUSED ? UB : 1][NCH][VEC];
  float v[UB];
  unsigned hbits;
  unsigned anew;   // FUSED: bit u set when a[u] holds a newly started row's A
};

template <typename T, int VEC, int LPN, int NCH, int UB, bool FUSED>
__device__ inline void load_batch(Batch<T, VEC, LPN, NCH, UB, FUSED>& bt, int64_t s0, int64_t b,
                                  int64_t ge, const int* s_col, const float* s_val,
                                  const uint64_t* s_head, const int* s_trow,
                                  const T* __restrict__ X, const T* __restrict__ A, int kz, int q,
                                  int nvec, int64_t gs, int lgS) {
  const bool any = s0 < ge;
  const int64_t sw = any ? s0 : b;   // a valid slot for the head word
  const int wi = (int)((sw - b) >> 6);
  const uint64_t hw = s_head[wi];
  bt.hbits = (unsigned)(hw >> (sw & 63)) & ((1u << UB) - 1u);
  int rbase = 0;
  if constexpr (FUSED) rbase = s_trow[wi] + __popcll(hw & lanemask_le((int)(sw & 63)) & ~1ull);
#pragma unroll
  for (int u = 0; u < UB; ++u) {
    const bool ok = s0 + u < ge;
    const int li0 = ok ? (int)(s0 - b) + u : 0;
    const int li = li0 + (li0 >> lgS);
    const int c = s_col[li];
    bt.v[u] = ok ? s_val[li] : 0.f;
    load_row<T, VEC, LPN, NCH>(X + (int64_t)c * kz, q, nvec, bt.x[u]);
    if constexpr (FUSED) {
      // one A access per row segment: at the group's first slot and where a
      // row starts
      const bool need = ok && (s0 + u == gs || (((bt.hbits >> u) & 1u) && s0 + u > gs));
      if (u == 0) bt.anew = 0;
      if (need) {
        const int r = rbase + __popc(bt.hbits & ((2u << u) - 1u) & ~1u);
        load_row<T, VEC, LPN, NCH>(A + (int64_t)r * kz, q, nvec, bt.a[u]);
        bt.anew |= 1u << u;
      }
    }
  }
}

// SpMM (and, with FUSED, SDDMM on the same pass: every slot's packed B row is
// read once and used both for the dot with its A row and for the row sum).
// SC (rows added into the owner's slab through Y.map): each row's destination
// values are loaded when the row starts, one row's map entry ahead, so the
// addition at the row's end issues a store instead of waiting for a load.
template <typename T, int VEC, int LPN, int NCH, bool FUSED, int UBT, bool SC = false>
__global__ __launch_bounds__(256) void k_spmm(int64_t nnz, int64_t nitems, int64_t nblocks,
                                              int wslots, const int32_t* __restrict__ idx,
                                              const uint64_t* __restrict__ head,
                                              const int32_t* __restrict__ tile_row,
                                              const float* __restrict__ vals,
                                              const int32_t* __restrict__ vidx,
                                              const T* __restrict__ X, int kz,
                                              YOut Y, int accumulate,
                                              float* __restrict__ carry, const T* __restrict__ A,
                                              float* __restrict__ out) {
  constexpr int G = 64 / LPN;
  constexpr int UB0 = UBT * (FUSED ? 2 : 4) / (NCH * VEC);
  constexpr int UB = UB0 < 1 ? 1 : (UB0 > UBT ? UBT : UB0);   // divides UBT (8 or 16)
  constexpr int KW = LPN * NCH * VEC;
  using BT = Batch<T, VEC, LPN, NCH, UB, FUSED>;
  extern __shared__ __align__(16) char smem[];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int g = lane / LPN, q = lane % LPN;
  const size_t P = (size_t)wslots + G;   // staged slots plus one pad word per run
  const int nwords = wslots / 64;
  const size_t wave_bytes = spmm_wave_lds(wslots, LPN, NCH, VEC, FUSED);
  char* wbase = smem + (size_t)wv * wave_bytes;
  // 8-byte head words first (wave_bytes is a multiple of 16)
  uint64_t* s_head = reinterpret_cast<uint64_t*>(wbase);
  char* wrest = wbase + (size_t)nwords * 8;
  int* s_col = reinterpret_cast<int*>(wrest);
  float* s_val = reinterpret_cast<float*>(wrest + P * 4);
  float* s_out = reinterpret_cast<float*>(wrest + P * 8);   // FUSED only
  float* s_lead = reinterpret_cast<float*>(wrest + P * (FUSED ? 12 : 8));
  int* s_kind = reinterpret_cast<int*>(wrest + P * (FUSED ? 12 : 8) + (size_t)G * KW * 4);
  int* s_trow = s_kind + G;

  const int64_t item = xcd_block(nblocks) * 4 + wv;
  const bool active = item < nitems;
  const int nvec = kz / VEC;
  const int S = wslots / G;
  const int lgS = __builtin_ctz(S);
  int64_t b = 0, e = 0;
  if (active) {
    b = item * wslots;
    e = (b + wslots < nnz) ? b + wslots : nnz;
    for (int i = lane; i < (int)(e - b); i += 64) {
      const int pi = i + (i >> lgS);
      s_col[pi] = ld_stream(idx + b + i);
      s_val[pi] = vals ? (vidx ? vals[vidx[b + i]] : ld_stream(vals + b + i)) : 1.f;
    }
    const int nw = (int)((e - b + 63) >> 6);   // b is a multiple of 64
    for (int i = lane; i < nw; i += 64) {
      s_head[i] = head[(b >> 6) + i];
      s_trow[i] = tile_row[(b >> 6) + i];
    }
  }
  __syncthreads();

  float acc[NCH][VEC];
  zero(acc);
  int kind = kLeadNone;
  bool tail = false, started = false;
  int cur = 0;
  const int64_t gs = b + (int64_t)g * S;
  const int64_t ge = (gs + S < e) ? gs + S : e;
  float pre[SC ? NCH : 1][VEC];   // SC: destination values of row cur
  float* ycur = nullptr;          // SC: destination row of cur
  int64_t gnext = 0;              // SC: map entry of row cur + 1
  if (active && gs < ge) {
    cur = row_of(head, tile_row, gs);
    started = is_head(head, gs);
    if constexpr (SC) {
      gnext = cur + 1 < Y.n ? Y.map[cur + 1] : 0;
      if (started) {
        ycur = Y.base + (Y.map[cur] - Y.lo) * Y.ld;
        load_dst<VEC, NCH>(ycur, nvec, q, LPN, pre);
      }
    }
    BT cb;
    float acur[FUSED ? NCH : 1][VEC];
    for (int64_t s0 = gs; s0 < ge; s0 += UB) {
      load_batch<T, VEC, LPN, NCH, UB, FUSED>(cb, s0, b, ge, s_col, s_val, s_head, s_trow, X, A,
                                              kz, q, nvec, gs, lgS);
      if constexpr (FUSED) {
#pragma unroll
        for (int u = 0; u < UB; ++u) {
          if ((cb.anew >> u) & 1u) {
#pragma unroll
            for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
              for (int t = 0; t < VEC; ++t) acur[ch][t] = cb.a[u][ch][t];
          }
          const float d = group_sum<LPN>(lane_dot<VEC, LPN, NCH>(acur, cb.x[u], q, nvec));
          const int li = (int)(s0 - b) + u;
          if (q == 0 && s0 + u < ge) s_out[li + (li >> lgS)] = cb.v[u] * d;
        }
      }
#pragma unroll
      for (int u = 0; u < UB; ++u) {
        if (s0 + u < ge) {
          if (s0 + u > gs && ((cb.hbits >> u) & 1u)) {
            if (started) {
              if constexpr (SC)
                store_pre<VEC, NCH>(ycur, nvec, q, LPN, pre, acc);
              else
                store_row<VEC, NCH>(Y, cur, kz, nvec, q, LPN, acc, accumulate);
            } else {
              store_vec<VEC, NCH>(s_lead + g * KW, nvec, q, LPN, acc);
              kind = kLeadEnds;
            }
            zero(acc);
            ++cur;
            started = true;
            if constexpr (SC) {
              ycur = Y.base + (gnext - Y.lo) * Y.ld;
              load_dst<VEC, NCH>(ycur, nvec, q, LPN, pre);
              gnext = cur + 1 < Y.n ? Y.map[cur + 1] : 0;
            }
          }
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int t = 0; t < VEC; ++t) acc[ch][t] = fmaf(cb.v[u], cb.x[u][ch][t], acc[ch][t]);
        }
      }
    }
    const bool ends = (ge >= nnz) || is_head(head, ge);
    if (started) {
      if (!ends)
        tail = true;
      else if constexpr (SC)
        store_pre<VEC, NCH>(ycur, nvec, q, LPN, pre, acc);
      else
        store_row<VEC, NCH>(Y, cur, kz, nvec, q, LPN, acc, accumulate);
    } else {
      store_vec<VEC, NCH>(s_lead + g * KW, nvec, q, LPN, acc);
      kind = ends ? kLeadEnds : kLeadThrough;
    }
  }
  if (q == 0) s_kind[g] = kind;
  __syncthreads();
  if (!active) return;

  if constexpr (FUSED) {
    for (int i = lane; i < (int)(e - b); i += 64)
      st_stream(out + b + i, (accumulate & kAccOut) ? ld_stream(out + b + i) + s_out[i + (i >> lgS)]
                                                    : s_out[i + (i >> lgS)]);
  }
  if (tail) {
    bool done = false;
    for (int g2 = g + 1; g2 < G; ++g2) {
      const int k = s_kind[g2];
      if (k == kLeadNone) break;
      add_vec<VEC, NCH>(s_lead + g2 * KW, nvec, q, LPN, acc);
      if (k == kLeadEnds) {
        done = true;
        break;
      }
    }
    if (!done)
      store_vec<VEC, NCH>(carry + (item * 2 + 1) * kz, nvec, q, LPN, acc);
    else if constexpr (SC)
      store_pre<VEC, NCH>(ycur, nvec, q, LPN, pre, acc);
    else
      store_row<VEC, NCH>(Y, cur, kz, nvec, q, LPN, acc, accumulate);
  }
  if (g == 0 && s_kind[0] != kLeadNone) {
    float hc[NCH][VEC];
    zero(hc);
    add_vec<VEC, NCH>(s_lead, nvec, q, LPN, hc);
    if (s_kind[0] == kLeadThrough) {
      for (int g2 = 1; g2 < G; ++g2) {
        const int k = s_kind[g2];
        if (k == kLeadNone) break;
        add_vec<VEC, NCH>(s_lead + g2 * KW, nvec, q, LPN, hc);
        if (k == kLeadEnds) break;
      }
    }
    store_vec<VEC, NCH>(carry + (item * 2) * kz, nvec, q, LPN, hc);
  }
}

// ------------------------------------------------- SpMM, windowed family
//
// The SDDMM window layout applied to SpMM: in each 64-slot window, group g
// owns slots g*L .. g*L+L-1 and has all their rows in flight at once (JB per
// batch), so a wavefront keeps as many rows in flight as the SDDMM kernel
// and needs no LDS.  Each lane sums s_p * X[col] over the group's slots in
// slot order; a row that starts and ends inside a group is stored directly.
// The pieces of rows that cross group boundaries meet in a segmented
// inclusive scan over the G groups (shuffles, log2 G steps, fixed order);
// the row running out of a window is carried in registers into the next.
// Rows cut by work-item boundaries leave head / tail carries for
// k_spmm_fixup, as the group-run family does.  With FUSED, the same rows
// also give the SDDMM dots (A rows loaded per slot, as in k_sddmm).
template <int VEC, int NCH>
__device__ inline void shfl_vec(const float (&src)[NCH][VEC], float (&dst)[NCH][VEC], int from) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
    for (int t = 0; t < VEC; ++t) dst[ch][t] = __shfl(src[ch][t], from);
}

__device__ inline int win_row(int trow, uint64_t hw, int i) {
  return trow + __popcll(hw & lanemask_le(i) & ~1ull);
}

template <typename T, int VEC, int LPN, int NCH, bool FUSED>
__global__ __launch_bounds__(256) void k_wspmm(int64_t nnz, int64_t nitems, int64_t nblocks,
                                               int wslots, const int32_t* __restrict__ idx,
                                               const uint64_t* __restrict__ head,
                                               const int32_t* __restrict__ tile_row,
                                               const float* __restrict__ vals,
                                               const int32_t* __restrict__ vidx,
                                               const T* __restrict__ X, int kz,
                                               YOut Y, int accumulate,
                                               float* __restrict__ carry,
                                               const T* __restrict__ A,
                                               float* __restrict__ out) {
  constexpr int G = 64 / LPN;
  constexpr int JB0 = FUSED ? 64 / (2 * NCH * VEC) : 64 / (NCH * VEC);
  constexpr int JB = JB0 < 1 ? 1 : (JB0 > LPN ? LPN : JB0);
  const int lane = threadIdx.x & 63;
  const int g = lane / LPN, q = lane % LPN;
  const int64_t item = xcd_block(nblocks) * 4 + (threadIdx.x >> 6);
  if (item >= nitems) return;   // uniform per wavefront; no barriers below
  const int nvec = kz / VEC;
  const int64_t b = item * wslots;
  const int64_t e = (b + wslots < nnz) ? b + wslots : nnz;
  const bool ends_at_e = (e >= nnz) || is_head(head, e);
  const int gl = g * LPN;

  float cy[NCH][VEC];   // the row running in from the previous window (same in every group)
  zero(cy);
  bool cy_own = false;  // that row started inside this item
  // The next window's indices, values and head word are loaded while the
  // current window's rows are in flight (one memory round trip per window).
  int col_n = 0;
  float v_n = 0.f;
  uint64_t hw_n = 0;
  int trow_n = 0;
  auto fetch = [&](int64_t w0) {
    const int64_t sl = w0 + lane;
    const bool ok = sl < e;
    col_n = ok ? ld_stream(idx + sl) : 0;
    v_n = ok ? (vals ? (vidx ? vals[vidx[sl]] : ld_stream(vals + sl)) : 1.f) : 0.f;
    hw_n = head[w0 >> 6];
    trow_n = tile_row[w0 >> 6];
  };
  fetch(b);
  for (int64_t win = b; win < e; win += 64) {
    const int nv = (e - win < 64) ? (int)(e - win) : 64;
    const bool valid = lane < nv;
    const int64_t sl = win + lane;
    const int col = col_n;
    const float v = v_n;
    uint64_t hw = hw_n;
    const int trow = trow_n;
    if (nv < 64) hw &= (1ull << nv) - 1ull;
    const bool more = win + 64 < e;
    const bool next_head = more ? (bool)(head[(win >> 6) + 1] & 1ull) : ends_at_e;
    if (more) fetch(win + 64);
    const bool g_head = (hw >> gl) & 1ull;

    float acc[NCH][VEC], lp[NCH][VEC];
    zero(acc);
    zero(lp);
    bool first_seg = true, has_lp = false;
    float res = 0.f;
#pragma unroll
    for (int j0 = 0; j0 < LPN; j0 += JB) {
      float bb[JB][NCH][VEC];
      float a[FUSED ? JB : 1][NCH][VEC];
      float sv[JB];
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const int src = gl + j0 + jj;
        const int c = __shfl(col, src);
        sv[jj] = __shfl(v, src);
        load_row<T, VEC, LPN, NCH>(X + (int64_t)c * kz, q, nvec, bb[jj]);
        if constexpr (FUSED)
          load_row<T, VEC, LPN, NCH>(A + (int64_t)win_row(trow, hw, src) * kz, q, nvec, a[jj]);
      }
#pragma unroll
      for (int jj = 0; jj < JB; ++jj) {
        const int j = j0 + jj, w = gl + j;
        if constexpr (FUSED) {
          const float d = group_sum<LPN>(lane_dot<VEC, LPN, NCH>(a[jj], bb[jj], q, nvec));
          if (q == j) res = d;
        }
        // A row starting at slot w ends the segment before it: a row complete
        // inside the group is stored; the group's first segment, when it began
        // in an earlier group, is kept for the scan.  Branch-free but the store.
        const bool in = w < nv;
        const bool brk = in && j > 0 && ((hw >> w) & 1ull);
        const bool to_lp = brk && first_seg && !g_head;
        if (brk && !to_lp)
          store_row<VEC, NCH>(Y, win_row(trow, hw, w - 1), kz, nvec, q, LPN, acc, accumulate);
#pragma unroll
        for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
          for (int t = 0; t < VEC; ++t) {
            lp[ch][t] = to_lp ? acc[ch][t] : lp[ch][t];
            const float a0 = brk ? 0.f : acc[ch][t];
            acc[ch][t] = in ? fmaf(sv[jj], bb[jj][ch][t], a0) : a0;
          }
        has_lp = has_lp || to_lp;
        first_seg = first_seg && !brk;
      }
    }
    if constexpr (FUSED) {
      if (valid) {
        const float o = v * res;
        st_stream(out + sl, (accumulate & kAccOut) ? ld_stream(out + sl) + o : o);
      }
    }

    // segmented inclusive scan of the groups' last segments
    bool f = !first_seg || g_head;   // this group's last segment starts in the group
    bool own = true;
    if (g == 0 && !f) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int t = 0; t < VEC; ++t) acc[ch][t] = cy[ch][t] + acc[ch][t];
      own = cy_own;
      f = true;
    }
#pragma unroll
    for (int d = 1; d < G; d <<= 1) {
      const int from = g >= d ? lane - d * LPN : lane;
      float xs[NCH][VEC];
      shfl_vec<VEC, NCH>(acc, xs, from);
      const bool fs = __shfl((int)f, from) != 0;
      const bool os = __shfl((int)own, from) != 0;
      if (g >= d) {
        if (!f) {
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
            for (int t = 0; t < VEC; ++t) acc[ch][t] = xs[ch][t] + acc[ch][t];
          own = os;
        }
        f = f || fs;
      }
    }
    // the row a group's first segment closes: the scan value of the group before
    float prev[NCH][VEC];
    shfl_vec<VEC, NCH>(acc, prev, g > 0 ? lane - LPN : lane);
    // (every shuffle runs on all 64 lanes: no shuffle reads an inactive lane)
    const bool own_left = __shfl((int)own, g > 0 ? lane - LPN : lane) != 0;
    const bool prev_own = g > 0 ? own_left : cy_own;
    if (g == 0) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int t = 0; t < VEC; ++t) prev[ch][t] = cy[ch][t];
    }
    if (has_lp) {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int t = 0; t < VEC; ++t) lp[ch][t] = prev[ch][t] + lp[ch][t];
      if (prev_own)
        store_row<VEC, NCH>(Y, win_row(trow, hw, gl), kz, nvec, q, LPN, lp, accumulate);
      else
        store_vec<VEC, NCH>(carry + (item * 2) * kz, nvec, q, LPN, lp);
    }
    // a row ending exactly at the end of a group inside the window
    const int glast = gl + LPN;
    if (g < G - 1 && glast < nv && ((hw >> glast) & 1ull)) {
      if (own)
        store_row<VEC, NCH>(Y, win_row(trow, hw, glast - 1), kz, nvec, q, LPN, acc, accumulate);
      else
        store_vec<VEC, NCH>(carry + (item * 2) * kz, nvec, q, LPN, acc);
    }
    // the row at the end of the window
    float last[NCH][VEC];
    shfl_vec<VEC, NCH>(acc, last, (G - 1) * LPN + q);
    const bool last_own = __shfl((int)own, (G - 1) * LPN) != 0;
    if (next_head || win + 64 >= e) {
      if (g == 0) {
        if (next_head) {
          if (last_own)
            store_row<VEC, NCH>(Y, win_row(trow, hw, nv - 1), kz, nvec, q, LPN, last, accumulate);
          else
            store_vec<VEC, NCH>(carry + (item * 2) * kz, nvec, q, LPN, last);
        } else {
          // the item ends inside a row: its owner finishes it in k_spmm_fixup
          store_vec<VEC, NCH>(carry + (item * 2 + (last_own ? 1 : 0)) * kz, nvec, q, LPN, last);
        }
      }
      zero(cy);
      cy_own = false;
    } else {
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int t = 0; t < VEC; ++t) cy[ch][t] = last[ch][t];
      cy_own = last_own;
    }
  }
}

// Rows cut by item boundaries: item j whose last row starts inside it and
// continues past its end owns the row; it adds its tail carry and the head
// carries of the items the row runs through, in item order.  One round of
// independent loads serves the common case (the row ends in item j + 1): the
// head words of items j and j + 1 and the first word of j + 2 (one per lane),
// the tile row of slot e - 1, j's tail carry and j + 1's head carry.  Only a
// row that runs past item j + 1 reads the row pointer and more carries.
template <int VEC, int LPN, int NCH>
__global__ __launch_bounds__(256) void k_spmm_fixup(int64_t nnz, int64_t nitems, int wslots,
                                                    const int32_t* __restrict__ ptr,
                                                    const uint64_t* __restrict__ head,
                                                    const int32_t* __restrict__ tile_row, int kz,
                                                    YOut Y, int accumulate,
                                                    const float* __restrict__ carry) {
  constexpr int G = 64 / LPN;
  constexpr int BLK = 16;
  const int lane = threadIdx.x & 63, g = lane / LPN, q = lane % LPN;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nitems) return;   // uniform per wavefront, as are the returns below
  const int64_t b = j * wslots, e = b + wslots;
  if (e >= nnz) return;      // the last item ends with the block
  const int nw = wslots >> 6;   // head words per item (wslots <= 1024: 2 nw + 1 <= 33 lanes)
  const int nvec = kz / VEC;
  const int64_t ntiles = (nnz + 63) >> 6;
  const int64_t wi = (b >> 6) + lane;
  const uint64_t hw = (lane <= 2 * nw && wi < ntiles) ? head[wi] : 0ull;
  const int trow = tile_row[(e - 1) >> 6];
  float tail[NCH][VEC], nxt[NCH][VEC];
  zero(tail);
  zero(nxt);
  add_vec<VEC, NCH>(carry + (j * 2 + 1) * kz, nvec, q, LPN, tail);
  add_vec<VEC, NCH>(carry + ((j + 1) * 2) * kz, nvec, q, LPN, nxt);
  if (__shfl(hw, nw) & 1ull) return;               // slot e starts a row
  if (!__any(lane < nw && hw != 0ull)) return;     // the row of slot e - 1 began before b
  const int r = trow + __popcll(__shfl(hw, nw - 1) & ~1ull);   // row of slot e - 1
  // the item holding the row's last slot: from the first row start after e
  const uint64_t found = __ballot(lane >= nw && lane <= 2 * nw && hw != 0ull);
  int64_t jl;
  if (found) {
    const int f = __ffsll((long long)found) - 1;
    const uint64_t wf = __shfl(hw, f);
    const int64_t sh = ((b >> 6) + f) * 64 + (__ffsll((long long)wf) - 1);
    jl = (sh - 1) / wslots;
  } else {
    jl = (e + wslots >= nnz) ? (nnz - 1) / wslots : ((int64_t)ptr[r + 1] - 1) / wslots;
  }
  float tot[NCH][VEC];
  if (jl == j + 1) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
      for (int t = 0; t < VEC; ++t) tot[ch][t] = nxt[ch][t];
  } else {
    zero(tot);
    for (int64_t j0 = j + 1 + g; j0 <= jl; j0 += (int64_t)G * BLK) {
      float blk[NCH][VEC];
      zero(blk);
      for (int m = 0; m < BLK; ++m) {
        const int64_t jj = j0 + (int64_t)m * G;
        if (jj > jl) break;
        add_vec<VEC, NCH>(carry + (jj * 2) * kz, nvec, q, LPN, blk);
      }
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int t = 0; t < VEC; ++t) tot[ch][t] += blk[ch][t];
    }
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1)
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int t = 0; t < VEC; ++t) tot[ch][t] += __shfl_xor(tot[ch][t], m * LPN);
  }
  if (g == 0) {
#pragma unroll
    for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
      for (int t = 0; t < VEC; ++t) tail[ch][t] += tot[ch][t];
    store_row<VEC, NCH>(Y, r, kz, nvec, q, LPN, tail, accumulate);
  }
}

// ------------------------------------------------------------ launch


struct Shape {
  int vec;    // elements per 16-byte load (1 = scalar path)
  int lanes;  // L
  int nch;    // vectors per lane
  int items;  // W
  int wide;   // SpMM: batches of up to 16 slots instead of 8
  int window; // SpMM: the windowed family (k_wspmm) instead of group runs
};

inline int pow2ceil(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

// op: 0 SDDMM, 1 SpMM, 2 fused SDDMM+SpMM.  Defaults (variant -1), from
// measurements on MI355X: SDDMM on 64-slot work items with lanes covering kz
// (8 lanes for 16-byte FP32 rows of 16 or more vectors below 2^20 entries); SpMM and
// the fused pass on work items that grow with the block, about nnz / 4096
// slots clamped to [64, 512] so that small blocks still launch enough
// wavefronts, in the windowed family below 2^18 entries (and below 2^20 for
// 16-byte rows of at most 4 vectors in the fused pass and FP32 SpMM) and in the
// group-run family above.  The fused pass holds A and B rows per batch; it
// takes half as many lanes for FP32 rows of 16 or more vectors (kz >= 64) and
// for bfloat16 rows of 16 vectors (kz = 128) from 2^18 entries on, where the
// smaller groups measured faster; other rows keep lanes covering the row.
// From 2^21 entries on, its 128-wide rows (FP32 and bfloat16) take work items
// of 256 slots instead of 512.
inline spc3d_status pick_shape(int kz, spc3d_dtype t, bool vec_ok, int variant, int op,
                               int64_t nnz, Shape* sh) {
  const bool spmm = op != 0;
  const int vfull = (t == SPC3D_F32) ? 4 : 8;
  sh->vec = (vec_ok && kz % vfull == 0) ? vfull : 1;
  if (sh->vec == 1 && kz > kMaxKzScalar)
    return fail(SPC3D_ERR_UNSUPPORTED, "kz=%d needs 16-byte aligned rows with kz %% %d == 0", kz,
                vfull);
  const int nvec = kz / sh->vec;
  if (variant < 0) {
    sh->lanes = pow2ceil(nvec);
    if (op == 2 && nvec >= 16 && (t == SPC3D_F32 || nnz >= (int64_t(1) << 18))) sh->lanes /= 2;
    if (op == 0 && t == SPC3D_F32 && sh->vec > 1 && nvec >= 16 && nnz < (int64_t(1) << 20))
      sh->lanes = 8;
    if (sh->lanes > 16) sh->lanes = 16;
    if (sh->lanes < 2) sh->lanes = 2;
    while ((nvec + sh->lanes - 1) / sh->lanes > 4) sh->lanes *= 2;
    sh->wide = 0;
    sh->window = 0;
    sh->items = 64;
    if (spmm) {
      sh->items = nnz < (int64_t(1) << 18) ? 64
                  : nnz < (int64_t(1) << 20) ? 128
                  : nnz < (int64_t(1) << 21) ? 256 : 512;
      if (op == 2 && kz == 128 && sh->items == 512) sh->items = 256;
      if (sh->items == 64 && sh->lanes <= 8)
        sh->window = 1;
      else if (sh->items == 128 && sh->lanes <= 4 && sh->vec > 1 && (op == 2 || t == SPC3D_F32))
        sh->window = 1;
      else
        while (sh->items / (64 / sh->lanes) < 8) sh->items *= 2;
    }
  } else {
    const int lg = variant & 15, lw = (variant >> 4) & 15;
    if (lg < 1 || lg > 6 || lw > 4 || (variant >> 10) || ((variant >> 8) & 3) == 3)
      return fail(SPC3D_ERR_INVALID_ARG, "bad variant %d", variant);
    sh->lanes = 1 << lg;
    sh->items = 64 << lw;
    sh->wide = (variant >> 8) & 1;
    sh->window = (variant >> 9) & 1;
  }
  sh->nch = (nvec + sh->lanes - 1) / sh->lanes;
  if (sh->nch == 3) sh->nch = 4;
  if (sh->nch > 4)
    return fail(SPC3D_ERR_UNSUPPORTED, "variant has too few lanes for kz=%d", kz);
  if (sh->window && spmm && sh->lanes > 8)
    return fail(SPC3D_ERR_UNSUPPORTED, "the windowed SpMM family takes 2, 4 or 8 lanes");
  if (spmm && !sh->window) {
    const int G = 64 / sh->lanes;
    if (sh->items / G < (sh->wide ? 16 : 8))
      return fail(SPC3D_ERR_UNSUPPORTED, "SpMM variant needs >= %d slots per group",
                  sh->wide ? 16 : 8);
  }
  return SPC3D_OK;
}

#define SPC3D_SWITCH_NCH(NCHV, ...)                     \
  switch (NCHV) {                                       \
    case 1: { constexpr int NCH_ = 1; __VA_ARGS__; break; } \
    case 2: { constexpr int NCH_ = 2; __VA_ARGS__; break; } \
    default: { constexpr int NCH_ = 4; __VA_ARGS__; break; } \
  }

#define SPC3D_SWITCH_LPN(LPNV, ...)                      \
  switch (LPNV) {                                        \
    case 2: { constexpr int LPN_ = 2; __VA_ARGS__; break; }  \
    case 4: { constexpr int LPN_ = 4; __VA_ARGS__; break; }  \
    case 8: { constexpr int LPN_ = 8; __VA_ARGS__; break; }  \
    case 16: { constexpr int LPN_ = 16; __VA_ARGS__; break; } \
    case 32: { constexpr int LPN_ = 32; __VA_ARGS__; break; } \
    default: { constexpr int LPN_ = 64; __VA_ARGS__; break; } \
  }

template <typename T, int VEC>
void launch_sddmm(const Shape& sh, hipStream_t st, int64_t nnz, int64_t nitems, int64_t nblocks,
                  const Orient& o, const float* vals, const void* A, const void* B, int kz,
                  float* out, int accumulate) {
  SPC3D_SWITCH_LPN(sh.lanes, SPC3D_SWITCH_NCH(sh.nch,
      hipLaunchKernelGGL((k_sddmm<T, VEC, LPN_, NCH_>), dim3((unsigned)nblocks), dim3(256), 0,
                         st, nnz, nitems, nblocks, sh.items, o.idx, o.head, o.tile_row, vals,
                         static_cast<const T*>(A), static_cast<const T*>(B), kz, out,
                         accumulate)));
}

template <typename T, int VEC, bool FUSED>
void launch_spmm(const Shape& sh, hipStream_t st, int64_t nnz, int64_t nitems, int64_t nblocks,
                 const Orient& o, const float* vals, const void* X, int kz, const YOut& Y,
                 int accumulate, float* carry, size_t lds, const void* A, float* out) {
  SPC3D_SWITCH_LPN(sh.lanes, SPC3D_SWITCH_NCH(sh.nch,
      if (sh.window) {
        // 2, 4 or 8 lanes (pick_shape); wider groups would unroll too far
        if constexpr (LPN_ <= 8)
          hipLaunchKernelGGL((k_wspmm<T, VEC, LPN_, NCH_, FUSED>), dim3((unsigned)nblocks),
                             dim3(256), 0, st, nnz, nitems, nblocks, sh.items, o.idx, o.head,
                             o.tile_row, vals, o.vidx, static_cast<const T*>(X), kz, Y,
                             accumulate, carry, static_cast<const T*>(A), out);
      } else if (sh.wide)
        hipLaunchKernelGGL((k_spmm<T, VEC, LPN_, NCH_, FUSED, 16>), dim3((unsigned)nblocks),
                           dim3(256), lds, st, nnz, nitems, nblocks, sh.items, o.idx, o.head,
                           o.tile_row, vals, o.vidx, static_cast<const T*>(X), kz, Y, accumulate,
                           carry, static_cast<const T*>(A), out);
      else if (FUSED && VEC % 4 == 0 && Y.map) {
        // rows added into the owner's slab: destination rows loaded ahead
        if constexpr (FUSED && VEC % 4 == 0)
          hipLaunchKernelGGL((k_spmm<T, VEC, LPN_, NCH_, FUSED, 8, true>),
                             dim3((unsigned)nblocks), dim3(256), lds, st, nnz, nitems, nblocks,
                             sh.items, o.idx, o.head, o.tile_row, vals, o.vidx,
                             static_cast<const T*>(X), kz, Y, accumulate, carry,
                             static_cast<const T*>(A), out);
      } else
        hipLaunchKernelGGL((k_spmm<T, VEC, LPN_, NCH_, FUSED, 8>), dim3((unsigned)nblocks),
                           dim3(256), lds, st, nnz, nitems, nblocks, sh.items, o.idx, o.head,
                           o.tile_row, vals, o.vidx, static_cast<const T*>(X), kz, Y, accumulate,
                           carry, static_cast<const T*>(A), out);
      hipLaunchKernelGGL((k_spmm_fixup<VEC, LPN_, NCH_>),
                         dim3((unsigned)((nitems + 3) / 4)), dim3(256), 0, st, nnz, nitems,
                         sh.items, o.ptr, o.head, o.tile_row, kz, Y, accumulate, carry)));
}

#define SPC3D_SDDMM_LAUNCH_ARGS                                                                \
  const Shape&, hipStream_t, int64_t, int64_t, int64_t, const Orient&, const float*, const void*, \
      const void*, int, float*, int
#define SPC3D_SPMM_LAUNCH_ARGS                                                                 \
  const Shape&, hipStream_t, int64_t, int64_t, int64_t, const Orient&, const float*, const void*, \
      int, const YOut&, int, float*, size_t, const void*, float*

}  // namespace spc3d
