// Plan checker: verifies on the device every local id that the compute,
// gather, scatter and permute kernels turn into an address, so that a plan
// whose arrays were overwritten (or a library bug in their construction) is
// reported as an error instead of becoming an out-of-bounds access.  The
// checked kernels themselves stay unchanged: spc3d_plan_check runs before
// them, on request or, with SPC3D_DEBUG_BOUNDS=1 in the environment, at the
// start of every call that launches them.
//
// Invariants (those the kernels rely on; the localization of Section "The
// setup phase" builds them):
//   rowptr[0] = 0, rowptr[R] = nnz, rowptr strictly increasing (every local
//   row holds an entry); colidx[s] in [0, C); head bit of slot s set exactly
//   when s = rowptr[r] for some r, and clear past nnz; tile_row[t] = the row
//   of slot 64t; perm[s] in [0, nnz); gmap_r[l] in [row_lo, row_hi) and
//   gmap_c[l] in [col_lo, col_hi), ascending unless the plan is
//   owner-grouped; and the same for the column-major arrays of a plan built
//   with SPC3D_BUILD_CSC (colptr, rowidx_t in [0, R), slot_t in [0, nnz),
//   head_t, tile_col).
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "internal.h"

namespace spc3d {
namespace {

enum CheckCode : int {
  kRowptrEnds = 1, kRowptrOrder, kColidx, kHead, kTileRow, kPerm, kGmapR, kGmapC,
  kColptrEnds, kColptrOrder, kRowidxT, kSlotT, kHeadT, kTileCol, kNumCodes
};

const char* code_name(int c) {
  switch (c) {
    case kRowptrEnds: return "rowptr[0] / rowptr[R]";
    case kRowptrOrder: return "rowptr not strictly increasing at row";
    case kColidx: return "colidx outside [0, C) at slot";
    case kHead: return "head bitmap disagrees with rowptr at slot";
    case kTileRow: return "tile_row wrong at tile";
    case kPerm: return "perm outside [0, nnz) at slot";
    case kGmapR: return "gmap_r outside the row range or out of order at local row";
    case kGmapC: return "gmap_c outside the column range or out of order at local column";
    case kColptrEnds: return "colptr[0] / colptr[C]";
    case kColptrOrder: return "colptr not strictly increasing at column";
    case kRowidxT: return "rowidx_t outside [0, R) at column-major slot";
    case kSlotT: return "slot_t outside [0, nnz) at column-major slot";
    case kHeadT: return "column-major head bitmap disagrees with colptr at slot";
    case kTileCol: return "tile_col wrong at tile";
  }
  return "unknown";
}

// The first violation found, as (code << 48) | index: the least code, then
// the least index, wins (atomicMin), so the report does not depend on timing.
static __device__ unsigned long long g_check_word;

__device__ inline void report(unsigned long long* w, int code, int64_t i) {
  const unsigned long long v =
      ((unsigned long long)code << 48) | ((unsigned long long)i & ((1ull << 48) - 1));
  atomicMin(w, v);
}

__global__ void k_check_reset(unsigned long long* w) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *w = ~0ull;
}

// Row of slot s: the largest r with ptr[r] <= s (binary search over ptr[0..n];
// reads stay inside ptr whatever its contents).
__device__ inline int64_t row_search(const int32_t* ptr, int64_t n, int64_t s) {
  int64_t a = 0, b = n;   // answer in [0, n)
  while (b - a > 1) {
    const int64_t m = (a + b) >> 1;
    if ((int64_t)ptr[m] <= s) a = m; else b = m;
  }
  return a;
}

// One orientation: ptr [n + 1], idx [nnz] in [0, nidx), head/tile over the
// nnz slots, val [nnz] (perm or slot_t) in [0, nnz).
__global__ void k_check_orient(int64_t nnz, int64_t n, int64_t nidx, const int32_t* ptr,
                               const int32_t* idx, const uint64_t* head, const int32_t* tile,
                               const int32_t* val, int c_ends, int c_order, int c_idx, int c_head,
                               int c_tile, int c_val, unsigned long long* w) {
  const int64_t ntiles = (nnz + 63) / 64;
  const int64_t total = nnz > n ? nnz : n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (i == 0 && (ptr[0] != 0 || (int64_t)ptr[n] != nnz)) report(w, c_ends, 0);
    if (i < n && ptr[i + 1] <= ptr[i]) report(w, c_order, i);
    if (i < nnz) {
      const int32_t c = idx[i];
      if (c < 0 || (int64_t)c >= nidx) report(w, c_idx, i);
      const int32_t v = val[i];
      if (v < 0 || (int64_t)v >= nnz) report(w, c_val, i);
      const bool bit = (head[i >> 6] >> (i & 63)) & 1ull;
      const bool start = (int64_t)ptr[row_search(ptr, n, i)] == i;
      if (bit != start) report(w, c_head, i);
    }
    if (i < ntiles) {
      if ((int64_t)tile[i] != row_search(ptr, n, 64 * i)) report(w, c_tile, i);
      const int64_t past = nnz - 64 * i;   // bits at or past nnz must be clear
      if (past < 64 && (head[i] >> past) != 0ull) report(w, c_head, 64 * i + past);
    }
  }
}

__global__ void k_check_gmap(int64_t n, const int64_t* gmap, int64_t lo, int64_t hi, int ordered,
                             int code, unsigned long long* w) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = gmap[i];
    if (g < lo || g >= hi || (ordered && i + 1 < n && gmap[i + 1] <= g)) report(w, code, i);
  }
}

unsigned grid_of(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (unsigned)b;
}

std::mutex g_word_mu;
void* g_word_addr[64] = {};

spc3d_status check_word(unsigned long long** out) {
  int dev = -1;
  SPC3D_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= 64) return fail(SPC3D_ERR_UNSUPPORTED, "device %d not served", dev);
  std::lock_guard<std::mutex> lk(g_word_mu);
  if (!g_word_addr[dev]) {
    void* a = nullptr;
    SPC3D_HIP(hipGetSymbolAddress(&a, HIP_SYMBOL(g_check_word)));
    if (!a) return fail(SPC3D_ERR_HIP, "no address for the check word");
    g_word_addr[dev] = a;
  }
  *out = static_cast<unsigned long long*>(g_word_addr[dev]);
  return SPC3D_OK;
}

}  // namespace

spc3d_status check_plan(Plan* p, hipStream_t stream) {
  DeviceGuard dg;
  spc3d_status st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  unsigned long long* w = nullptr;
  st = check_word(&w);
  if (st != SPC3D_OK) return st;
  hipLaunchKernelGGL(k_check_reset, dim3(1), dim3(64), 0, stream, w);
  const bool grouped = p->ngroups_r > 0 || p->ngroups_c > 0;
  hipLaunchKernelGGL(k_check_gmap, dim3(grid_of(p->R)), dim3(256), 0, stream, p->R, p->gmap_r,
                     p->row_lo, p->row_hi, grouped ? 0 : 1, (int)kGmapR, w);
  hipLaunchKernelGGL(k_check_gmap, dim3(grid_of(p->C)), dim3(256), 0, stream, p->C, p->gmap_c,
                     p->col_lo, p->col_hi, grouped ? 0 : 1, (int)kGmapC, w);
  if (p->nnz > 0) {
    const int64_t nr = p->nnz > p->R ? p->nnz : p->R;
    hipLaunchKernelGGL(k_check_orient, dim3(grid_of(nr)), dim3(256), 0, stream, p->nnz, p->R,
                       p->C, p->rowptr, p->colidx, p->head, p->tile_row, p->perm,
                       (int)kRowptrEnds, (int)kRowptrOrder, (int)kColidx, (int)kHead,
                       (int)kTileRow, (int)kPerm, w);
    if (p->flags & SPC3D_BUILD_CSC) {
      const int64_t nc = p->nnz > p->C ? p->nnz : p->C;
      hipLaunchKernelGGL(k_check_orient, dim3(grid_of(nc)), dim3(256), 0, stream, p->nnz, p->C,
                         p->R, p->colptr, p->rowidx_t, p->head_t, p->tile_col, p->slot_t,
                         (int)kColptrEnds, (int)kColptrOrder, (int)kRowidxT, (int)kHeadT,
                         (int)kTileCol, (int)kSlotT, w);
    }
  }
  SPC3D_LAUNCHED("plan_check");
  unsigned long long word = 0;
  SPC3D_HIP(hipMemcpyAsync(&word, w, sizeof word, hipMemcpyDeviceToHost, stream));
  SPC3D_HIP(hipStreamSynchronize(stream));
  if (word == ~0ull) return SPC3D_OK;
  const int code = (int)(word >> 48);
  const long long at = (long long)(word & ((1ull << 48) - 1));
  return fail(SPC3D_ERR_OUT_OF_RANGE, "plan check failed: %s %lld", code_name(code), at);
}

namespace {
bool debug_on() {
  static const bool on = [] {
    const char* e = std::getenv("SPC3D_DEBUG_BOUNDS");
    return e && *e && std::strcmp(e, "0") != 0;
  }();
  return on;
}
}  // namespace

spc3d_status debug_check(Plan* p, hipStream_t stream) {
  return debug_on() ? check_plan(p, stream) : SPC3D_OK;
}

}  // namespace spc3d

using namespace spc3d;

extern "C" {

spc3d_status spc3d_plan_check(spc3d_plan h, hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  return check_plan(p, stream);
}

int spc3d_debug_bounds(void) { return debug_on() ? 1 : 0; }

}  // extern "C"
