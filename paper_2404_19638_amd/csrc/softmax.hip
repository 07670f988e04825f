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
};

enum { kNone = 0, kEnds = 1, kThrough = 2 };

__device__ inline int row_of_slot(const uint64_t* __restrict__ head,
                                  const int32_t* __restrict__ tile_row, int64_t s) {
  return tile_row[s >> 6] + __popcll(head[s >> 6] & lanemask_le((int)(s & 63)) & ~1ull);
}

__device__ inline bool head_at(const uint64_t* __restrict__ head, int64_t s) {
  return (head[s >> 6] >> (s & 63)) & 1ull;
}

// stats[r] = reduction of row r for rows inside one item; carries for the rest.
template <class Op>
__global__ __launch_bounds__(256) void k_row_reduce(int64_t nnz, int64_t nitems, int wslots,
                                                    const uint64_t* __restrict__ head,
                                                    const int32_t* __restrict__ tile_row,
                                                    const float* __restrict__ x0,
                                                    const float* __restrict__ x1,
                                                    typename Op::St* __restrict__ stats,
                                                    typename Op::St* __restrict__ carry) {
  using St = typename Op::St;
  __shared__ St s_lead[4][64];
  __shared__ int s_kind[4][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t item = (int64_t)blockIdx.x * 4 + wv;
  const bool active = item < nitems;
  const int S = wslots / 64;
  int64_t b = 0, e = 0;
  if (active) {
    b = item * wslots;
    e = (b + wslots < nnz) ? b + wslots : nnz;
  }
  const int64_t gs = b + (int64_t)lane * S;
  const int64_t ge = (gs + S < e) ? gs + S : e;
  St acc = Op::init();
  int kind = kNone, cur = 0;
  bool started = false, tail = false;
  if (active && gs < ge) {
    cur = row_of_slot(head, tile_row, gs);
    started = head_at(head, gs);
    for (int64_t s = gs; s < ge; ++s) {
      if (s > gs && head_at(head, s)) {
        if (started) {
          stats[cur] = acc;
        } else {
          s_lead[wv][lane] = acc;
          kind = kEnds;
        }
        acc = Op::init();
        ++cur;
        started = true;
      }
      Op::push(acc, Op::input(x0, x1, s));
    }
    const bool ends = (ge >= nnz) || head_at(head, ge);
    if (started) {
      if (ends)
        stats[cur] = acc;
      else
        tail = true;
    } else {
      s_lead[wv][lane] = acc;
      kind = ends ? kEnds : kThrough;
    }
  }
  s_kind[wv][lane] = kind;
  __syncthreads();
  if (!active) return;
  if (tail) {
    bool done = false;
    for (int l2 = lane + 1; l2 < 64; ++l2) {
      const int k = s_kind[wv][l2];
      if (k == kNone) break;
      acc = Op::merge(acc, s_lead[wv][l2]);
      if (k == kEnds) {
        done = true;
        break;
      }
    }
    if (done)
      stats[cur] = acc;
    else
      carry[item * 2 + 1] = acc;
  }
  if (lane == 0 && s_kind[wv][0] != kNone) {
    St hc = s_lead[wv][0];
    if (s_kind[wv][0] == kThrough) {
      for (int l2 = 1; l2 < 64; ++l2) {
        const int k = s_kind[wv][l2];
        if (k == kNone) break;
        hc = Op::merge(hc, s_lead[wv][l2]);
        if (k == kEnds) break;
      }
    }
    carry[item * 2] = hc;
  }
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

__global__ void k_softmax_apply(int64_t nnz, const uint64_t* __restrict__ head,
                                const int32_t* __restrict__ tile_row,
                                const SoftmaxStat::St* __restrict__ stats,
                                const float* __restrict__ e, float* __restrict__ alpha) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    const SoftmaxStat::St st = stats[row_of_slot(head, tile_row, p)];
    alpha[p] = expf(e[p] - st.m) / st.s;
  }
}

__global__ void k_softmax_bwd_apply(int64_t nnz, const uint64_t* __restrict__ head,
                                    const int32_t* __restrict__ tile_row,
                                    const DotSum::St* __restrict__ stats,
                                    const float* __restrict__ alpha,
                                    const float* __restrict__ dalpha, float* __restrict__ de) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    const float d = stats[row_of_slot(head, tile_row, p)].s;
    de[p] = alpha[p] * (dalpha[p] - d);
  }
}

__global__ void k_mul_values(int64_t n, const float* __restrict__ a, const float* __restrict__ b,
                             float* __restrict__ out) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < n;
       p += (int64_t)gridDim.x * blockDim.x)
    out[p] = a[p] * b[p];
}

namespace {

constexpr int kRowItems = 256;   // slots per wavefront work item (4 per lane)

size_t softmax_buffer_bytes(const Plan* p) {
  const int64_t nitems = (p->nnz + kRowItems - 1) / kRowItems;
  return (size_t)(p->R > 0 ? p->R : 1) * 8 + ((size_t)(nitems > 0 ? nitems : 1) * 2) * 8 + 256;
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
  hipLaunchKernelGGL(k_row_reduce<Op>, dim3(nb), dim3(256), 0, stream, p->nnz, nitems,
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
  st = use_device(p);
  if (st != SPC3D_OK) return st;
  SoftmaxStat::St* stats;
  st = row_reduce<SoftmaxStat>(p, d_e, nullptr, d_buf, stream, &stats);
  if (st != SPC3D_OK) return st;
  hipLaunchKernelGGL(k_softmax_apply, dim3(blocks_for(p->nnz)), dim3(256), 0, stream, p->nnz,
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
  st = use_device(p);
  if (st != SPC3D_OK) return st;
  DotSum::St* stats;
  st = row_reduce<DotSum>(p, d_alpha, d_dalpha, d_buf, stream, &stats);
  if (st != SPC3D_OK) return st;
  hipLaunchKernelGGL(k_softmax_bwd_apply, dim3(blocks_for(p->nnz)), dim3(256), 0, stream,
                     p->nnz, p->head, p->tile_row, stats, d_alpha, d_dalpha, d_de);
  SPC3D_LAUNCHED("softmax bwd apply");
  return SPC3D_OK;
}

spc3d_status spc3d_mul_values(spc3d_plan h, const float* d_a, const float* d_b, float* d_out,
                              hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_a || !d_b || !d_out) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  st = use_device(p);
  if (st != SPC3D_OK) return st;
  hipLaunchKernelGGL(k_mul_values, dim3(blocks_for(p->nnz)), dim3(256), 0, stream, p->nnz, d_a,
                     d_b, d_out);
  SPC3D_LAUNCHED("mul_values");
  return SPC3D_OK;
}

}  // extern "C"
