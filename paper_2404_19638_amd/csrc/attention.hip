// Fused masked attention forward over a localized block (an extension built
// on the paper's two kernels, not part of the paper).  For every stored entry
// p of local row i with column j:
//
//   score  e_p     = <q_i, k_j>                          (SDDMM, Eq. (1), s == 1)
//   weight alpha_p = exp(e_p - m_i) / s_i,  m_i = max of row i's scores,
//                    s_i = sum over row i of exp(e_q - m_i)
//   output out_i   = sum_p alpha_p v_j                   (SpMM, Eq. (2))
//
// in one pass over the block, so neither the scores nor the weights are
// written to memory (the SDDMM -> softmax -> SpMM fusion the paper's related
// work calls FusedMM).  Each row segment keeps a running triple (m, s, a): the
// largest score so far, the sum of exp(e - m) and the sum of exp(e - m) v.  A
// new score e costs one exponential: when e > m the sums so far are rescaled
// by exp(m - e) and e becomes the maximum, otherwise exp(e - m) is added.  Two
// partial triples of one row merge by rescaling both to the larger maximum.
// At the row's end out_i = a / s, and (m_i, s_i) are stored so that the
// backward pass can rebuild alpha from recomputed scores.
//
// Work decomposition.  Group g (LPN lanes) of a wavefront owns the contiguous
// run of S = 2^lg_s slots [b + g*S, b + (g+1)*S) of its work item (S <= 64,
// so a run lies inside one 64-bit head word), walked in steps of U slots.
// Lane q holds the column index of slot q % 4 of each step and DPP quad
// broadcasts hand slot u's index to its whole group; the U key and value rows
// of a step (and the query rows of the rows that start in it) are loaded as
// raw 16-byte vectors before any is used.  Row triples are finished where the
// next row starts; the part of a row before a run's first row start and the
// part after its last meet in a segmented suffix scan over the groups
// (shuffles, log2 G steps), and rows cut by work-item boundaries leave head /
// tail carries that k_attn_fixup merges in a fixed order.  All merge orders
// depend only on the structure, so results are deterministic.
#include <cmath>

#include "kernels.h"

namespace spc3d {

template <int NCH, int VEC>
struct Tri {
  float m, s;
  float a[NCH][VEC];
};

template <int NCH, int VEC>
__device__ inline void tri_init(Tri<NCH, VEC>& t) {
  t.m = -INFINITY;
  t.s = 0.f;
  zero(t.a);
}

// x <- x (+) y: both rescaled to the larger maximum (equal maxima, including
// two empty triples, scale by exactly 1).
template <int NCH, int VEC>
__device__ inline void tri_merge(Tri<NCH, VEC>& x, const Tri<NCH, VEC>& y) {
  const float m = fmaxf(x.m, y.m);
  const float cx = (x.m == m) ? 1.f : expf(x.m - m);
  const float cy = (y.m == m) ? 1.f : expf(y.m - m);
  x.s = fmaf(x.s, cx, y.s * cy);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
    for (int k = 0; k < VEC; ++k) x.a[ch][k] = fmaf(x.a[ch][k], cx, y.a[ch][k] * cy);
  x.m = m;
}

// Adds score e with value row v (one exponential).
template <int NCH, int VEC>
__device__ inline void tri_push(Tri<NCH, VEC>& t, float e, const float (&v)[NCH][VEC]) {
  const bool up = e > t.m;
  const float x = (e == t.m) ? 1.f : expf(-fabsf(e - t.m));
  const float c = up ? x : 1.f;
  const float p = up ? 1.f : x;
  t.s = fmaf(t.s, c, p);
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
    for (int k = 0; k < VEC; ++k) t.a[ch][k] = fmaf(t.a[ch][k], c, p * v[ch][k]);
  t.m = up ? e : t.m;
}

template <int NCH, int VEC>
__device__ inline void tri_shfl(const Tri<NCH, VEC>& t, Tri<NCH, VEC>& o, int from) {
  o.m = __shfl(t.m, from);
  o.s = __shfl(t.s, from);
  shfl_vec<VEC, NCH>(t.a, o.a, from);
}

// Carry record of kz + 4 floats: the kz weighted sums, then m and s.
template <int LPN, int NCH, int VEC>
__device__ inline void tri_store(float* __restrict__ rec, int kz, int nvec, int q,
                                 const Tri<NCH, VEC>& t) {
  store_vec<VEC, NCH>(rec, nvec, q, LPN, t.a);
  if (q == 0) {
    rec[kz] = t.m;
    rec[kz + 1] = t.s;
  }
}

template <int LPN, int NCH, int VEC>
__device__ inline void tri_load(const float* __restrict__ rec, int kz, int nvec, int q,
                                Tri<NCH, VEC>& t) {
  zero(t.a);
  add_vec<VEC, NCH>(rec, nvec, q, LPN, t.a);
  t.m = rec[kz];
  t.s = rec[kz + 1];
}

// out row i = a / s; stats[2i] = m, stats[2i+1] = s.
template <int LPN, int NCH, int VEC>
__device__ inline void tri_finish(float* __restrict__ out, float* __restrict__ stats, int64_t row,
                                  int kz, int nvec, int q, const Tri<NCH, VEC>& t) {
  float o[NCH][VEC];
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
    for (int k = 0; k < VEC; ++k) o[ch][k] = t.a[ch][k] / t.s;
  store_row<VEC, NCH>(out, row, kz, nvec, q, LPN, o, 0);
  if (stats && q == 0) {
    stats[2 * row] = t.m;
    stats[2 * row + 1] = t.s;
  }
}

template <typename T, int VEC, int LPN, int NCH>
__device__ inline void load_raw(const T* __restrict__ row, int q, uint4 (&r)[NCH]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) r[ch] = *reinterpret_cast<const uint4*>(row + (q + ch * LPN) * VEC);
}

template <typename T, int VEC, int NCH>
__device__ inline void unpack_row(const uint4 (&r)[NCH], float (&o)[NCH][VEC]) {
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) Unpack<T, VEC>::run(r[ch], o[ch]);
}

// Lane u of this lane's group (groups of 4 or more lanes: lane u of the own
// quad, which holds the same slot).
__device__ inline int quad_bcast(int v, int u) {
  switch (u) {
    case 0: return __builtin_amdgcn_update_dpp(0, v, 0x00, 0xF, 0xF, false);
    case 1: return __builtin_amdgcn_update_dpp(0, v, 0x55, 0xF, 0xF, false);
    case 2: return __builtin_amdgcn_update_dpp(0, v, 0xAA, 0xF, 0xF, false);
    default: return __builtin_amdgcn_update_dpp(0, v, 0xFF, 0xF, 0xF, false);
  }
}

// Lanes of a group cover the row exactly: LPN * NCH * VEC == kz.
template <typename T, int VEC, int LPN, int NCH, int U>
__global__ __launch_bounds__(256) void k_attn_fwd(int64_t nnz, int64_t nitems, int64_t nblocks,
                                                  int lg_s, const int32_t* __restrict__ idx,
                                                  const uint64_t* __restrict__ head,
                                                  const int32_t* __restrict__ tile_row,
                                                  const T* __restrict__ Q,
                                                  const T* __restrict__ Kf,
                                                  const T* __restrict__ V, int kz,
                                                  float* __restrict__ out,
                                                  float* __restrict__ stats,
                                                  float* __restrict__ carry) {
  static_assert(LPN >= 4 && LPN <= 16 && U >= 1 && U <= 4, "attention shape");
  using Tr = Tri<NCH, VEC>;
  constexpr int G = 64 / LPN;
  const int lane = threadIdx.x & 63, g = lane / LPN, q = lane % LPN;
  const int64_t item = xcd_block(nblocks) * 4 + (threadIdx.x >> 6);
  if (item >= nitems) return;   // uniform per wavefront; no barriers below
  const int S = 1 << lg_s;
  const int64_t W = (int64_t)G << lg_s;
  const int64_t b = item * W;
  const int64_t e = (b + W < nnz) ? b + W : nnz;
  const int64_t gs = b + ((int64_t)g << lg_s);
  const int nrun = gs >= e ? 0 : (e - gs < S ? (int)(e - gs) : S);
  const int nvec = kz / VEC;
  const int CS = kz + 4;
  const bool ends_at_e = (e >= nnz) || is_head(head, e);

  // head bits of the run (bit t: slot gs + t starts a row) and the row of gs
  const int64_t gw = (gs < nnz ? gs : nnz - 1) >> 6;
  const uint64_t hword = head[gw];
  const int sh = (int)(gs & 63);
  const uint64_t vmask = nrun >= 64 ? ~0ull : ((1ull << nrun) - 1ull);
  const uint64_t run = (hword >> sh) & vmask;
  const int rbase = tile_row[gw] + __popcll(hword & lanemask_le(sh) & ~1ull);

  const int qq = q & 3;   // slot of each step whose index this lane holds
  auto col_of = [&](int m) {
    const int t = m * U + (qq < U ? qq : 0);
    const int c = ld_stream(idx + (t < nrun ? gs + t : 0));
    return t < nrun ? c : 0;
  };

  Tr cur, lead;
  tri_init(cur);
  tri_init(lead);
  float qv[NCH][VEC];
  zero(qv);
  bool seen = run & 1ull;
  int r = rbase;
  const int steps = S / U;
  int cn = col_of(0);
  for (int m = 0; m < steps; ++m) {
    const int cc = cn;
    if (m + 1 < steps) cn = col_of(m + 1);
    const unsigned hb = (unsigned)(run >> (m * U)) & ((1u << U) - 1u);
    uint4 kr[U][NCH], vr[U][NCH], qr[U][NCH];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int c = quad_bcast(cc, u);
      load_raw<T, VEC, LPN, NCH>(Kf + (int64_t)c * kz, q, kr[u]);
      load_raw<T, VEC, LPN, NCH>(V + (int64_t)c * kz, q, vr[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = m * U + u;
      if (t < nrun && (t == 0 || ((hb >> u) & 1u))) {
        const int ru = rbase + __popcll(run & ((2ull << t) - 1ull) & ~1ull);
        load_raw<T, VEC, LPN, NCH>(Q + (int64_t)ru * kz, q, qr[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int t = m * U + u;
      const bool valid = t < nrun;
      const bool starts = valid && (t == 0 || ((hb >> u) & 1u));
      if (starts) unpack_row<T, VEC, NCH>(qr[u], qv);
      float kx[NCH][VEC];
      unpack_row<T, VEC, NCH>(kr[u], kx);
      float d = 0.f;
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch)
#pragma unroll
        for (int k = 0; k < VEC; ++k) d = fmaf(qv[ch][k], kx[ch][k], d);
      const float score = group_sum<LPN>(d);
      if (starts && t > 0) {
        if (seen)
          tri_finish<LPN, NCH, VEC>(out, stats, r, kz, nvec, q, cur);
        else
          lead = cur;
        tri_init(cur);
        ++r;
        seen = true;
      }
      if (valid) {
        float vx[NCH][VEC];
        unpack_row<T, VEC, NCH>(vr[u], vx);
        tri_push(cur, score, vx);
      }
    }
  }

  // (P, f): the run's lead (the whole run when no row starts in it) and
  // whether a row starts in the run.  Suffix scan over the groups:
  // Sv_g = P_g (+) Sv_{g+1} unless f_g;  F_g = f_g | F_{g+1}.
  const bool f = seen;
  Tr sv = f ? lead : cur;
  bool F = f;
#pragma unroll
  for (int d = 1; d < G; d <<= 1) {
    const bool inr = g + d < G;
    const int src = inr ? lane + d * LPN : lane;
    Tr o;
    tri_shfl(sv, o, src);
    const bool of = __shfl((int)F, src) != 0;
    if (inr && !F) tri_merge(sv, o);
    F = F || (inr && of);
  }
  const bool has_next = g + 1 < G;
  const int nsrc = has_next ? lane + LPN : lane;
  Tr nx;
  tri_shfl(sv, nx, nsrc);
  const bool nF = (__shfl((int)F, nsrc) != 0) && has_next;
  if (f) {
    // the run's last row: its tail and the leads of the runs it continues into
    if (has_next) tri_merge(cur, nx);
    if (nF || ends_at_e)
      tri_finish<LPN, NCH, VEC>(out, stats, r, kz, nvec, q, cur);
    else
      tri_store<LPN, NCH, VEC>(carry + (item * 2 + 1) * CS, kz, nvec, q, cur);
  }
  // the item starts inside a row: its head carry for the row's owner
  if (g == 0 && nrun > 0 && !(run & 1ull))
    tri_store<LPN, NCH, VEC>(carry + (item * 2) * CS, kz, nvec, q, sv);
}

// Rows cut by item boundaries: item j whose last row starts inside it and
// runs past its end owns the row; it merges its tail carry with the head
// carries of the items the row runs through (blocked per group, then a
// butterfly over the groups: a fixed order).
template <int VEC, int LPN, int NCH>
__global__ __launch_bounds__(256) void k_attn_fixup(int64_t nnz, int64_t nitems, int64_t wslots,
                                                    const int32_t* __restrict__ ptr,
                                                    const uint64_t* __restrict__ head,
                                                    const int32_t* __restrict__ tile_row, int kz,
                                                    float* __restrict__ out,
                                                    float* __restrict__ stats,
                                                    const float* __restrict__ carry) {
  using Tr = Tri<NCH, VEC>;
  constexpr int G = 64 / LPN;
  constexpr int BLK = 16;
  const int lane = threadIdx.x & 63, g = lane / LPN, q = lane % LPN;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (j >= nitems) return;
  const int64_t b = j * wslots, e = b + wslots;
  if (e >= nnz || is_head(head, e)) return;
  const int r = row_of(head, tile_row, e - 1);
  if (ptr[r] < b) return;
  const int64_t jl = ((int64_t)ptr[r + 1] - 1) / wslots;
  const int nvec = kz / VEC;
  const int CS = kz + 4;
  Tr tot;
  tri_init(tot);
  for (int64_t j0 = j + 1 + g; j0 <= jl; j0 += (int64_t)G * BLK) {
    Tr blk;
    tri_init(blk);
    for (int m = 0; m < BLK; ++m) {
      const int64_t jj = j0 + (int64_t)m * G;
      if (jj > jl) break;
      Tr c;
      tri_load<LPN, NCH, VEC>(carry + (jj * 2) * CS, kz, nvec, q, c);
      tri_merge(blk, c);
    }
    tri_merge(tot, blk);
  }
#pragma unroll
  for (int m = G / 2; m >= 1; m >>= 1) {
    Tr o;
    tri_shfl(tot, o, lane ^ (m * LPN));
    tri_merge(tot, o);
  }
  if (g == 0) {
    Tr res;
    tri_load<LPN, NCH, VEC>(carry + (j * 2 + 1) * CS, kz, nvec, q, res);
    tri_merge(res, tot);
    tri_finish<LPN, NCH, VEC>(out, stats, r, kz, nvec, q, res);
  }
}

namespace {

struct AttnShape {
  int vec, lanes, nch, u, lg_s;
};

// variant: -1, or lg_lanes (bits 0-3, 2..4) | lg_s << 4 (4..6).
spc3d_status attn_shape(int32_t kz, spc3d_dtype t, int variant, AttnShape* sh) {
  sh->vec = t == SPC3D_F32 ? 4 : 8;
  if (kz % sh->vec != 0)
    return fail(SPC3D_ERR_UNSUPPORTED, "fused attention needs kz %% %d == 0 (kz=%d)", sh->vec, kz);
  const int nvec = kz / sh->vec;
  if (variant < 0) {
    // measured on MI355X (R-MAT 2^16..2^20, K = 64): runs of 64 slots
    sh->lanes = nvec < 16 ? nvec : 16;
    sh->lg_s = 6;
  } else {
    const int lg = variant & 15, lgs = (variant >> 4) & 15;
    if (lg < 2 || lg > 4 || lgs < 4 || lgs > 6 || (variant >> 8))
      return fail(SPC3D_ERR_INVALID_ARG, "bad attention variant %d", variant);
    sh->lanes = 1 << lg;
    sh->lg_s = lgs;
  }
  if (sh->lanes < 4 || nvec % sh->lanes != 0 || nvec / sh->lanes > 2 ||
      (sh->lanes & (sh->lanes - 1)))
    return fail(SPC3D_ERR_UNSUPPORTED, "fused attention does not cover kz=%d with %d lanes", kz,
                sh->lanes);
  sh->nch = nvec / sh->lanes;
  sh->u = sh->nch == 1 ? 4 : 2;
  return SPC3D_OK;
}

int64_t attn_items(const Plan* p, const AttnShape& sh) {
  const int64_t W = (int64_t)(64 / sh.lanes) << sh.lg_s;
  return (p->nnz + W - 1) / W;
}

template <typename T, int VEC>
void launch_attn(const AttnShape& sh, hipStream_t st, const Plan* p, int64_t nitems,
                 const void* Q, const void* K, const void* V, int kz, float* out, float* stats,
                 float* carry) {
  const int64_t nblocks = (nitems + 3) / 4;
  const int64_t W = (int64_t)(64 / sh.lanes) << sh.lg_s;
  const T* q = static_cast<const T*>(Q);
  const T* k = static_cast<const T*>(K);
  const T* v = static_cast<const T*>(V);
#define SPC3D_ATTN(LPN, NCH, U)                                                                  \
  do {                                                                                         \
    hipLaunchKernelGGL((k_attn_fwd<T, VEC, LPN, NCH, U>), dim3((unsigned)nblocks), dim3(256), 0, \
                       st, p->nnz, nitems, nblocks, sh.lg_s, p->colidx, p->head, p->tile_row, q, \
                       k, v, kz, out, stats, carry);                                           \
    hipLaunchKernelGGL((k_attn_fixup<VEC, LPN, NCH>), dim3((unsigned)((nitems + 3) / 4)),      \
                       dim3(256), 0, st, p->nnz, nitems, W, p->rowptr, p->head, p->tile_row, kz, \
                       out, stats, carry);                                                     \
  } while (0)
  if (sh.nch == 1) {
    if (sh.lanes == 4) SPC3D_ATTN(4, 1, 4);
    else if (sh.lanes == 8) SPC3D_ATTN(8, 1, 4);
    else SPC3D_ATTN(16, 1, 4);
  } else {
    if (sh.lanes == 4) SPC3D_ATTN(4, 2, 2);
    else if (sh.lanes == 8) SPC3D_ATTN(8, 2, 2);
    else SPC3D_ATTN(16, 2, 2);
  }
#undef SPC3D_ATTN
}

}  // namespace
}  // namespace spc3d

using namespace spc3d;

extern "C" {

spc3d_status spc3d_attention_fwd_buffer_size(spc3d_plan h, int32_t kz, spc3d_dtype t, int variant,
                                             size_t* bytes) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (!bytes) return fail(SPC3D_ERR_INVALID_ARG, "bytes is NULL");
  if (t != SPC3D_F32 && t != SPC3D_BF16) return fail(SPC3D_ERR_INVALID_ARG, "bad dtype");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "kz=%d outside [1,%d]", kz, kMaxKz);
  AttnShape sh;
  st = attn_shape(kz, t, variant, &sh);
  if (st != SPC3D_OK) return st;
  const int64_t nitems = attn_items(p, sh);
  *bytes = (size_t)(nitems > 0 ? nitems : 1) * 2 * (size_t)(kz + 4) * 4;
  return SPC3D_OK;
}

spc3d_status spc3d_attention_fwd(spc3d_plan h, const void* d_Q, const void* d_K, const void* d_V,
                                 spc3d_dtype t, int32_t kz, float* d_out, float* d_stats,
                                 int variant, void* d_buf, size_t buf_bytes, hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (t != SPC3D_F32 && t != SPC3D_BF16) return fail(SPC3D_ERR_INVALID_ARG, "bad dtype");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "kz=%d outside [1,%d]", kz, kMaxKz);
  AttnShape sh;
  st = attn_shape(kz, t, variant, &sh);
  if (st != SPC3D_OK) return st;
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_Q || !d_K || !d_V || !d_out || !d_buf) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  if (!aligned16(d_Q) || !aligned16(d_K) || !aligned16(d_V) || !aligned16(d_out))
    return fail(SPC3D_ERR_INVALID_ARG, "Q, K, V and out must be 16-byte aligned");
  if (d_stats && (reinterpret_cast<uintptr_t>(d_stats) & 7u))
    return fail(SPC3D_ERR_INVALID_ARG, "stats must be 8-byte aligned");
  if (reinterpret_cast<uintptr_t>(d_buf) & 255u)
    return fail(SPC3D_ERR_INVALID_ARG, "buffer must be 256-byte aligned");
  const int64_t nitems = attn_items(p, sh);
  const size_t need = (size_t)nitems * 2 * (size_t)(kz + 4) * 4;
  if (buf_bytes < need)
    return fail(SPC3D_ERR_WORKSPACE, "attention buffer %zu bytes < %zu required", buf_bytes, need);
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
  float* carry = static_cast<float*>(d_buf);
  if (t == SPC3D_F32)
    launch_attn<float, 4>(sh, stream, p, nitems, d_Q, d_K, d_V, kz, d_out, d_stats, carry);
  else
    launch_attn<bf16_t, 8>(sh, stream, p, nitems, d_Q, d_K, d_V, kz, d_out, d_stats, carry);
  SPC3D_LAUNCHED("attention_fwd");
  return SPC3D_OK;
}

}  // extern "C"
