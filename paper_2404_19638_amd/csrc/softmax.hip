// Row-wise softmax over the stored entries of each row and its backward, the
// step between SDDMM edge scores and SpMM aggregation in a graph-attention
// layer (an extension built on the paper's two kernels, not part of the
// paper).
//
// Forward:  alpha_p = exp(e_p - m_r) / sum_{q in row r} exp(e_q - m_r),
//           m_r the row maximum.
// Backward: de_p = alpha_p * (dalpha_p - sum_{q in row r} alpha_q dalpha_q).
//
// Both are a per-row reduction followed by a per-slot map.  The reduction
// uses the same slot-split work items as SpMM (W slots per wavefront, here one
// lane per run of W/64 slots), so hub rows are spread over many wavefronts:
// the forward keeps an online (max, sum of exp) pair per row segment and
// merges pairs with the usual rescaling; the backward keeps a plain sum.
// Rows cut by item boundaries are finished by a fix-up pass in item order.
#include <cmath>

#include "internal.h"

namespace spc3d {

struct SoftmaxStat {
  struct St {
    float m, s;
  };
  static __device__ inline St init() { return {-INFINITY, 0.f}; }
  static __device__ inline void push(St& a, float x) {
    if (x > a.m) {
      a.s = a.s * expf(a.m - x) + 1.f;
      a.m = x;
    } else {
      a.s += expf(x - a.m);
    }
  }
  static __device__ inline St merge(St a, St b) {
    if (b.s == 0.f) return a;
    if (a.s == 0.f) return b;
    const float m = fmaxf(a.m, b.m);
    return {m, a.s * expf(a.m - m) + b.s * expf(b.m - m)};
  }
  static __device__ inline float input(const float* x0, const float*, int64_t p) { return x0[p]; }
  template <int N>
  static __device__ inline void loadv(const float* x0, const float*, int64_t p, float (&x)[N]) {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      const float4 v = *reinterpret_cast<const float4*>(x0 + p + i);
      x[i] = v.x; x[i + 1] = v.y; x[i + 2] = v.z; x[i + 3] = v.w;
    }
  }
};

struct DotSum {
  struct St {
    float m, s;   // m unused
  };
  static __device__ inline St init() { return {0.f, 0.f}; }
  static __device__ inline void push(St& a, float x) { a.s += x; }
  static __device__ inline St merge(St a, St b) { return {0.f, a.s + b.s}; }
  static __device__ inline float input(const float* x0, const float* x1, int64_t p) {
    return x0[p] * x1[p];
  }
  template <int N>
  static __device__ inline void loadv(const float* x0, const float* x1, int64_t p, float (&x)[N]) {
#pragma unroll
    for (int i = 0; i < N; i += 4) {
      const float4 a = *reinterpret_cast<const float4*>(x0 + p + i);
      const float4 b = *reinterpret_cast<const float4*>(x1 + p + i);
      x[i] = a.x * b.x; x[i + 1] = a.y * b.y; x[i + 2] = a.z * b.z; x[i + 3] = a.w * b.w;
    }
  }
};

__device__ inline int row_of_slot(const uint64_t* __restrict__ head,
                                  const int32_t* __restrict__ tile_row, int64_t s) {
  return tile_row[s >> 6] + __popcll(head[s >> 6] & lanemask_le((int)(s & 63)) & ~1ull);
}

__device__ inline bool head_at(const uint64_t* __restrict__ head, int64_t s) {
  return (head[s >> 6] >> (s & 63)) & 1ull;
}

// stats[r] = reduction of row r for rows inside one item; carries for the rest.
// Each lane owns a run of kRun consecutive slots; the run's head word, its
// inputs (kRun / 4 16-byte loads per input array where aligned) and the head
// bit after the item are loaded before any is used.  Runs of 16 measured
// faster than 8 or 4: half as many wavefronts, more bytes in flight each.  Rows that start and end in
// a run are written directly; the part of a row before a run's first row
// start ("lead") and the part after its last ("tail") meet in a segmented
// suffix scan over the 64 lanes (shuffles, 6 steps, a fixed order): lane l's
// tail row continues through the leads of lanes l+1, l+2, ... up to the first
// lane in which a row starts.
constexpr int kRun = 16;

template <class Op>
__device__ inline typename Op::St shfl_st(typename Op::St v, int from) {
  typename Op::St o;
  o.m = __shfl(v.m, from);
  o.s = __shfl(v.s, from);
  return o;
}

template <class Op, bool VEC4>
__global__ __launch_bounds__(256) void k_row_reduce(int64_t nnz, int64_t nitems, int wslots,
                                                    const uint64_t* __restrict__ head,
                                                    const int32_t* __restrict__ tile_row,
                                                    const float* __restrict__ x0,
                                                    const float* __restrict__ x1,
                                                    typename Op::St* __restrict__ stats,
                                                    typename Op::St* __restrict__ carry) {
  using St = typename Op::St;
  const int lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (item >= nitems) return;   // uniform per wavefront; no barriers below
  const int64_t b = item * wslots;
  const int64_t e = (b + wslots < nnz) ? b + wslots : nnz;
  const int64_t gs = b + (int64_t)lane * kRun;   // wslots == 64 * kRun
  const int n = gs < e ? (e - gs < kRun ? (int)(e - gs) : kRun) : 0;
  const bool ends_at_e = (e >= nnz) || head_at(head, e);
  St acc = Op::init(), lead = Op::init();
  bool seen = false;
  unsigned bits = 0;
  int cur = 0;
  if (n > 0) {
    float x[kRun];
    if (VEC4 && n == kRun) {
      Op::template loadv<kRun>(x0, x1, gs, x);
    } else {
#pragma unroll
      for (int i = 0; i < kRun; ++i) x[i] = i < n ? Op::input(x0, x1, gs + i) : 0.f;
    }
    const uint64_t hw = head[gs >> 6];
    const int sh = (int)(gs & 63);
    bits = (unsigned)(hw >> sh) & ((1u << n) - 1u);   // n <= kRun <= 16
    cur = tile_row[gs >> 6] + __popcll(hw & lanemask_le(sh) & ~1ull);
    seen = bits & 1u;
#pragma unroll
    for (int i = 0; i < kRun; ++i) {
      if (i < n) {
        if (i > 0 && ((bits >> i) & 1u)) {
          if (seen)
            stats[cur] = acc;
          else
            lead = acc;
          acc = Op::init();
          ++cur;
          seen = true;
        }
        Op::push(acc, x[i]);
      }
    }
  }
  // (P, f): the lane's lead (its whole run when no row starts in it) and
  // whether a row starts in it.  Sv_l = P_l (+) Sv_{l+1} unless f_l.
  St sv = seen ? lead : acc;
  bool F = seen;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const bool inr = lane + d < 64;
    const int src = inr ? lane + d : lane;
    const St o = shfl_st<Op>(sv, src);
    const bool of = __shfl((int)F, src) != 0;
    if (inr && !F) sv = Op::merge(sv, o);
    F = F || (inr && of);
  }
  const int nsrc = lane < 63 ? lane + 1 : lane;
  const St nx = shfl_st<Op>(sv, nsrc);
  const bool nF = (__shfl((int)F, nsrc) != 0) && lane < 63;
  if (seen) {
    if (lane < 63) acc = Op::merge(acc, nx);
    if (nF || ends_at_e)
      stats[cur] = acc;
    else
      carry[item * 2 + 1] = acc;
  }
  if (lane == 0 && n > 0 && !(bits & 1u)) carry[item * 2] = sv;
}

template <class Op>
__global__ __launch_bounds__(256) void k_row_reduce_fixup(int64_t nnz, int64_t nitems, int wslots,
                                                          const int32_t* __restrict__ ptr,
                                                          const uint64_t* __restrict__ head,
                                                          const int32_t* __restrict__ tile_row,
                                                          typename Op::St* __restrict__ stats,
                                                          const typename Op::St* __restrict__ carry) {
  using St = typename Op::St;
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nitems) return;
  const int64_t b = j * wslots, e = b + wslots;
  if (e >= nnz || head_at(head, e)) return;
  const int r = row_of_slot(head, tile_row, e - 1);
  if (ptr[r] < b) return;
  const int64_t jl = ((int64_t)ptr[r + 1] - 1) / wslots;
  St acc = Op::init();
  for (int64_t jj = j + 1 + lane; jj <= jl; jj += 64) acc = Op::merge(acc, carry[jj * 2]);
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    St o;
    o.m = __shfl_xor(acc.m, m);
    o.s = __shfl_xor(acc.s, m);
    acc = Op::merge(acc, o);
  }
  if (lane == 0) stats[r] = Op::merge(carry[j * 2 + 1], acc);
}

// The per-entry maps.  A wavefront takes kApplyWin consecutive 64-slot
// windows per iteration (grid-stride); lane i takes slot i of each, so every
// access to the per-entry arrays is coalesced, and the windows' loads are
// issued together: two waits per 64 * kApplyWin slots (head words and inputs,
// then row stats).  Eight windows measured 2-3% faster than four.
constexpr int kApplyWin = 8;

template <class Op>
__device__ inline void apply_windows(int64_t nnz, const uint64_t* __restrict__ head,
                                     const int32_t* __restrict__ tile_row,
                                     const typename Op::St* __restrict__ stats,
                                     const float* __restrict__ x0, const float* __restrict__ x1,
                                     float* __restrict__ y) {
  const int lane = threadIdx.x & 63;
  const int64_t nwin = (nnz + 63) >> 6;
  const int64_t ngrp = (nwin + kApplyWin - 1) / kApplyWin;
  for (int64_t gi = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); gi < ngrp;
       gi += (int64_t)gridDim.x * 4) {
    int row[kApplyWin];
    float a[kApplyWin], da[kApplyWin];
#pragma unroll
    for (int k = 0; k < kApplyWin; ++k) {
      const int64_t w = gi * kApplyWin + k;
      const int64_t wc = w < nwin ? w : nwin - 1;
      const int64_t p = wc * 64 + lane;
      const int64_t pc = p < nnz ? p : nnz - 1;
      row[k] = tile_row[wc] + __popcll(head[wc] & lanemask_le(lane) & ~1ull);
      a[k] = x0[pc];
      da[k] = x1 ? x1[pc] : 0.f;
    }
#pragma unroll
    for (int k = 0; k < kApplyWin; ++k) {
      const int64_t p = (gi * kApplyWin + k) * 64 + lane;
      const typename Op::St st = stats[row[k]];
      if (p < nnz) y[p] = Op::apply(a[k], da[k], st);
    }
  }
}

struct SoftmaxApply {
  using St = SoftmaxStat::St;
  static __device__ inline float apply(float e, float, St st) { return expf(e - st.m) / st.s; }
};

struct SoftmaxBwdApply {
  using St = DotSum::St;
  static __device__ inline float apply(float a, float da, St st) { return a * (da - st.s); }
};

__global__ __launch_bounds__(256) void k_softmax_apply(int64_t nnz,
                                                       const uint64_t* __restrict__ head,
                                                       const int32_t* __restrict__ tile_row,
                                                       const SoftmaxStat::St* __restrict__ stats,
                                                       const float* __restrict__ e,
                                                       float* __restrict__ alpha) {
  apply_windows<SoftmaxApply>(nnz, head, tile_row, stats, e, nullptr, alpha);
}

__global__ __launch_bounds__(256) void k_softmax_bwd_apply(int64_t nnz,
                                                           const uint64_t* __restrict__ head,
                                                           const int32_t* __restrict__ tile_row,
                                                           const DotSum::St* __restrict__ stats,
                                                           const float* __restrict__ alpha,
                                                           const float* __restrict__ dalpha,
                                                           float* __restrict__ de) {
  apply_windows<SoftmaxBwdApply>(nnz, head, tile_row, stats, alpha, dalpha, de);
}

__global__ void k_mul_values(int64_t n, const float* __restrict__ a, const float* __restrict__ b,
                             float* __restrict__ out) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    out[p] = a[p] * b[p];
}

namespace {

constexpr int kRowItems = 64 * kRun;   // slots per wavefront work item (kRun per lane)
static_assert(kRowItems == 64 * kRun, "one run per lane");

size_t softmax_buffer_bytes(const Plan* p) {
  const int64_t nitems = (p->nnz + kRowItems - 1) / kRowItems;
  return (size_t)(p->R > 0 ? p->R : 1) * 8 + ((size_t)(nitems > 0 ? nitems : 1) * 2) * 8 + 256;
}

// Workgroups for the apply kernels: one wavefront per kApplyWin windows.
unsigned apply_blocks(int64_t nnz) {
  const int64_t waves = ((nnz + 63) / 64 + kApplyWin - 1) / kApplyWin;
  int64_t b = (waves + 3) / 4;
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (unsigned)b;
}

unsigned blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (unsigned)b;
}

template <class Op>
spc3d_status row_reduce(const Plan* p, const float* x0, const float* x1, void* buf,
                        hipStream_t stream, typename Op::St** stats_out) {
  using St = typename Op::St;
  const int64_t nitems = (p->nnz + kRowItems - 1) / kRowItems;
  St* stats = static_cast<St*>(buf);
  const size_t off = (((size_t)(p->R > 0 ? p->R : 1) * 8) + 255) & ~size_t(255);
  St* carry = reinterpret_cast<St*>(static_cast<char*>(buf) + off);
  const unsigned nb = (unsigned)((nitems + 3) / 4);
  // 16-byte loads of each lane's run where the arrays allow them
  if (aligned16(x0) && (!x1 || aligned16(x1)))
    hipLaunchKernelGGL((k_row_reduce<Op, true>), dim3(nb), dim3(256), 0, stream, p->nnz, nitems,
                       kRowItems, p->head, p->tile_row, x0, x1, stats, carry);
  else
    hipLaunchKernelGGL((k_row_reduce<Op, false>), dim3(nb), dim3(256), 0, stream, p->nnz, nitems,
                       kRowItems, p->head, p->tile_row, x0, x1, stats, carry);
  hipLaunchKernelGGL(k_row_reduce_fixup<Op>, dim3(nb), dim3(256), 0, stream, p->nnz, nitems,
                     kRowItems, p->rowptr, p->head, p->tile_row, stats, carry);
  SPC3D_LAUNCHED("row reduce");
  *stats_out = stats;
  return SPC3D_OK;
}

}  // namespace
}  // namespace spc3d

using namespace spc3d;

extern "C" {

spc3d_status spc3d_row_softmax_buffer_size(spc3d_plan h, size_t* bytes) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (!bytes) return fail(SPC3D_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = softmax_buffer_bytes(p) + 256;
  return SPC3D_OK;
}

spc3d_status spc3d_row_softmax(spc3d_plan h, const float* d_e, float* d_alpha, void* d_buf,
                               size_t buf_bytes, hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_e || !d_alpha || !d_buf) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_buf) & 255u)
    return fail(SPC3D_ERR_INVALID_ARG, "buffer must be 256-byte aligned");
  if (buf_bytes < softmax_buffer_bytes(p))
    return fail(SPC3D_ERR_WORKSPACE, "softmax buffer too small");
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
  SoftmaxStat::St* stats;
  st = row_reduce<SoftmaxStat>(p, d_e, nullptr, d_buf, stream, &stats);
  if (st != SPC3D_OK) return st;
  hipLaunchKernelGGL(k_softmax_apply, dim3(apply_blocks(p->nnz)), dim3(256), 0, stream, p->nnz,
                     p->head, p->tile_row, stats, d_e, d_alpha);
  SPC3D_LAUNCHED("softmax apply");
  return SPC3D_OK;
}

spc3d_status spc3d_row_softmax_bwd(spc3d_plan h, const float* d_alpha, const float* d_dalpha,
                                   float* d_de, void* d_buf, size_t buf_bytes,
                                   hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_alpha || !d_dalpha || !d_de || !d_buf)
    return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_buf) & 255u)
    return fail(SPC3D_ERR_INVALID_ARG, "buffer must be 256-byte aligned");
  if (buf_bytes < softmax_buffer_bytes(p))
    return fail(SPC3D_ERR_WORKSPACE, "softmax buffer too small");
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
  DotSum::St* stats;
  st = row_reduce<DotSum>(p, d_alpha, d_dalpha, d_buf, stream, &stats);
  if (st != SPC3D_OK) return st;
  hipLaunchKernelGGL(k_softmax_bwd_apply, dim3(apply_blocks(p->nnz)), dim3(256), 0, stream,
                     p->nnz, p->head, p->tile_row, stats, d_alpha, d_dalpha, d_de);
  SPC3D_LAUNCHED("softmax bwd apply");
  return SPC3D_OK;
}

spc3d_status spc3d_row_softmax_apply(spc3d_plan h, const float* d_e, const float* d_stats,
                                     float* d_alpha, hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_e || !d_stats || !d_alpha) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_stats) & 7u)
    return fail(SPC3D_ERR_INVALID_ARG, "stats must be 8-byte aligned");
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
  hipLaunchKernelGGL(k_softmax_apply, dim3(apply_blocks(p->nnz)), dim3(256), 0, stream, p->nnz,
                     p->head, p->tile_row, reinterpret_cast<const SoftmaxStat::St*>(d_stats), d_e,
                     d_alpha);
  SPC3D_LAUNCHED("softmax apply");
  return SPC3D_OK;
}

spc3d_status spc3d_mul_values(spc3d_plan h, const float* d_a, const float* d_b, float* d_out,
                              hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_a || !d_b || !d_out) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
  hipLaunchKernelGGL(k_mul_values, dim3(blocks_for(p->nnz)), dim3(256), 0, stream, p->nnz, d_a,
                     d_b, d_out);
  SPC3D_LAUNCHED("mul_values");
  return SPC3D_OK;
}

}  // extern "C"
