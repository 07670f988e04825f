// Setup phase: localization of a sparse block (globalMap / localMap, empty
// rows and columns removed) and construction of its row-major and optional
// column-major slot structure.  Paper: Section "Data distribution" (localized
// blocks and the two maps) and Section "General structure" (a setup phase run
// once per sparsity pattern, after which iterations only move data).
//
// Device pipeline, all HBM-streaming:
//   mark ids      flag[g - lo] = 1 for every id (range violations raise a flag)
//   scan flags    lmap[g - lo] = exclusive prefix or -1; gmap[rank] = g
//   key/value     key = lr << bits(C) | lc, value = caller index
//   radix sort    LSD, 8-bit digits, stable (so equal keys keep caller order)
//   build slots   colidx, perm, rowptr, per-64-slot head bitmaps and tile rows
// and the same sort again on (lc, lr) for the column-major view.
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <unordered_set>

#include "internal.h"

namespace spc3d {

// ------------------------------------------------------------- errors

static thread_local std::string g_last_error;

spc3d_status fail(spc3d_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

spc3d_status hip_fail(hipError_t e, const char* what) {
  return fail(SPC3D_ERR_HIP, "%s: %s", what, hipGetErrorString(e));
}

static std::mutex g_plans_mu;
static std::unordered_set<const void*> g_plans;

spc3d_status get_plan(spc3d_plan h, Plan** out) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  if (!h || !g_plans.count(static_cast<const void*>(h)))
    return fail(SPC3D_ERR_BAD_HANDLE, "not a live plan");
  Plan* p = reinterpret_cast<Plan*>(h);
  if (p->magic != kPlanMagic) return fail(SPC3D_ERR_BAD_HANDLE, "corrupt plan");
  *out = p;
  return SPC3D_OK;
}

spc3d_status DeviceGuard::enter(const Plan* p) {
  int cur = -1;
  SPC3D_HIP(hipGetDevice(&cur));
  if (cur != p->device) {
    SPC3D_HIP(hipSetDevice(p->device));
    prev_ = cur;
  }
  return SPC3D_OK;
}

// ------------------------------------------------------------- kernels

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;   // 4096

__device__ inline int wave_inclusive_sum(int v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    int t = __shfl_up(v, d, 64);
    if (lane >= d) v += t;
  }
  return v;
}

// Exclusive prefix of v over the block (NT threads); *total gets the sum.
template <int NT>
__device__ inline int block_exclusive_sum(int v, int* total) {
  __shared__ int wsum[NT / 64];
  const int inc = wave_inclusive_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 63) wsum[w] = inc;
  __syncthreads();
  int off = 0, tot = 0;
#pragma unroll
  for (int i = 0; i < NT / 64; ++i) {
    int s = wsum[i];
    off += (i < w) ? s : 0;
    tot += s;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void k_mark(int64_t nnz, const int64_t* __restrict__ gid, int64_t lo, int64_t hi,
                       int32_t* __restrict__ flag, int32_t* __restrict__ err) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = gid[p];
    if (g < lo || g >= hi) {
      err[0] = 1;
    } else {
      flag[g - lo] = 1;
    }
  }
}

// Block sums of in[] over tiles of kScanTile.
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const int32_t* __restrict__ in,
                                                              int64_t n,
                                                              int32_t* __restrict__ partial) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t j = base + (int64_t)i * kScanThreads + threadIdx.x;
    s += (j < n) ? in[j] : 0;
  }
  int tot;
  block_exclusive_sum<kScanThreads>(s, &tot);
  if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// Exclusive scan of partial[0..m) in place by one block; total -> *total.
__global__ __launch_bounds__(1024) void k_scan_partials(int32_t* partial, int64_t m,
                                                        int32_t* total) {
  int carry = 0;
  for (int64_t base = 0; base < m; base += 1024) {
    int64_t j = base + threadIdx.x;
    int v = (j < m) ? partial[j] : 0;
    int tot;
    int ex = block_exclusive_sum<1024>(v, &tot);
    if (j < m) partial[j] = carry + ex;
    carry += tot;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

// Blocked per-thread prefix within a tile: thread t owns items
// [t*kScanItems, (t+1)*kScanItems) of the tile.
struct TileScan {
  int v[kScanItems];
  int ex[kScanItems];
};

__device__ inline void tile_exclusive(const int32_t* __restrict__ in, int64_t n, int64_t base,
                                      int offset, TileScan& ts) {
  int s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t j = base + (int64_t)threadIdx.x * kScanItems + i;
    ts.v[i] = (j < n) ? in[j] : 0;
    s += ts.v[i];
  }
  int tot;
  int ex = block_exclusive_sum<kScanThreads>(s, &tot) + offset;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    ts.ex[i] = ex;
    ex += ts.v[i];
  }
}

__global__ __launch_bounds__(kScanThreads) void k_scan_down(const int32_t* in, int64_t n,
                                                            const int32_t* __restrict__ partial,
                                                            int32_t* out) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  TileScan ts;
  tile_exclusive(in, n, base, partial[blockIdx.x], ts);
  __syncthreads();   // in and out may alias
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t j = base + (int64_t)threadIdx.x * kScanItems + i;
    if (j < n) out[j] = ts.ex[i];
  }
}

// Flags -> localMap (rank or -1) and globalMap (rank -> global id).
__global__ __launch_bounds__(kScanThreads) void k_compact(int32_t* lmap, int64_t n, int64_t lo,
                                                          const int32_t* __restrict__ partial,
                                                          int64_t* __restrict__ gmap) {
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  TileScan ts;
  tile_exclusive(lmap, n, base, partial[blockIdx.x], ts);
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    int64_t j = base + (int64_t)threadIdx.x * kScanItems + i;
    if (j < n) {
      if (ts.v[i]) {
        lmap[j] = ts.ex[i];
        gmap[ts.ex[i]] = lo + j;
      } else {
        lmap[j] = -1;
      }
    }
  }
}

__global__ void k_make_keys(int64_t nnz, const int64_t* __restrict__ rgid,
                            const int64_t* __restrict__ cgid, int64_t rlo, int64_t clo,
                            const int32_t* __restrict__ lmap_r, const int32_t* __restrict__ lmap_c,
                            int bits_c, uint64_t* __restrict__ key, int32_t* __restrict__ val) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t lr = (uint32_t)lmap_r[rgid[p] - rlo];
    const uint64_t lc = (uint32_t)lmap_c[cgid[p] - clo];
    key[p] = (lr << bits_c) | lc;
    val[p] = (int32_t)p;
  }
}

// Keys of the column-major view from the row-major slots: (lc << bits_r) | lr,
// value = row-major slot.
__global__ void k_make_keys_t(int64_t nnz, const uint64_t* __restrict__ skey, int bits_c,
                              int bits_r, uint64_t* __restrict__ key, int32_t* __restrict__ val) {
  const uint64_t cmask = bits_c ? ((1ull << bits_c) - 1ull) : 0ull;
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t k = skey[p];
    key[p] = ((k & cmask) << bits_r) | (k >> bits_c);
    val[p] = (int32_t)p;
  }
}

// ---------------------------------------------------------- radix sort

constexpr int kSortThreads = 256;
constexpr int kSortRounds = 8;
constexpr int kSortTile = kSortThreads * kSortRounds;   // 2048 keys per block

__global__ __launch_bounds__(kSortThreads) void k_radix_hist(const uint64_t* __restrict__ key,
                                                             int64_t n, int shift, int64_t nblk,
                                                             int32_t* __restrict__ counts) {
  __shared__ int hist[256];
  hist[threadIdx.x] = 0;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    int64_t j = base + r * kSortThreads + threadIdx.x;
    if (j < n) atomicAdd(&hist[(key[j] >> shift) & 255], 1);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * nblk + blockIdx.x] = hist[threadIdx.x];
}

// Stable scatter of one tile of kSortTile keys.  Items are ranked in rounds
// of 256 (item r*256 + t of the tile), so the rank of an item among equal
// digits follows tile order.  Each item is first placed in LDS at its
// position inside the tile's digit-ordered sequence; the tile is then
// written out in that order, so consecutive threads store consecutive
// elements of one digit's run instead of one element per cache line.
__global__ __launch_bounds__(kSortThreads) void k_radix_scatter(
    const uint64_t* __restrict__ kin, const int32_t* __restrict__ vin, int64_t n, int shift,
    int64_t nblk, const int32_t* __restrict__ offsets, uint64_t* __restrict__ kout,
    int32_t* __restrict__ vout) {
  __shared__ uint64_t s_key[kSortTile];
  __shared__ int32_t s_val[kSortTile];
  __shared__ int start[256];   // first position of each digit inside the tile
  __shared__ int cnt[256];     // items of each digit in the tile
  __shared__ int base[256];    // next free position of each digit (advances per round)
  __shared__ int wcnt[kSortThreads / 64][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t tile = (int64_t)blockIdx.x * kSortTile;
  uint64_t k[kSortRounds];
  int32_t v[kSortRounds];
  cnt[t] = 0;
  for (int i = 0; i < kSortThreads / 64; ++i) wcnt[i][t] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t j = tile + r * kSortThreads + t;
    k[r] = j < n ? kin[j] : 0;
    v[r] = j < n ? vin[j] : 0;
    if (j < n) atomicAdd(&cnt[(int)((k[r] >> shift) & 255)], 1);
  }
  __syncthreads();
  int total;
  const int st = block_exclusive_sum<kSortThreads>(cnt[t], &total);
  start[t] = st;
  base[t] = st;
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
#pragma unroll
  for (int r = 0; r < kSortRounds; ++r) {
    const int64_t j = tile + r * kSortThreads + t;
    const bool valid = j < n;
    const int d = (int)((k[r] >> shift) & 255);
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t bb = __ballot((d >> bit) & 1);
      peers &= ((d >> bit) & 1) ? bb : ~bb;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[w][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int pos = base[d] + rank;
      for (int i = 0; i < w; ++i) pos += wcnt[i][d];
      s_key[pos] = k[r];
      s_val[pos] = v[r];
    }
    __syncthreads();
    int add = 0;
    for (int i = 0; i < kSortThreads / 64; ++i) {
      add += wcnt[i][t];
      wcnt[i][t] = 0;
    }
    base[t] += add;
    __syncthreads();
  }
  // positions [0, total) of the tile now hold its items in (digit, tile order)
  for (int i = t; i < total; i += kSortThreads) {
    const uint64_t key = s_key[i];
    const int d = (int)((key >> shift) & 255);
    const int within = i - start[d];
    if (within < 0 || within >= cnt[d]) continue;   // cannot happen; keeps stores in range
    const int64_t g = (int64_t)offsets[(int64_t)d * nblk + blockIdx.x] + within;
    if (g < n) {
      kout[g] = key;
      vout[g] = s_val[i];
    }
  }
}

// Sorted keys -> slot arrays.  One thread per slot; lanes of a wavefront hold
// 64 consecutive slots, so the head bitmap word is one ballot.
__global__ __launch_bounds__(256) void k_build_slots(int64_t nnz, int64_t nrows,
                                                     const uint64_t* __restrict__ key,
                                                     const int32_t* __restrict__ val, int bits_minor,
                                                     int32_t* __restrict__ minor_out,
                                                     int32_t* __restrict__ val_out,
                                                     int32_t* __restrict__ ptr,
                                                     uint64_t* __restrict__ head,
                                                     int32_t* __restrict__ tile_row) {
  const int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const uint64_t mmask = bits_minor ? ((1ull << bits_minor) - 1ull) : 0ull;
  const bool valid = s < nnz;
  bool is_head = false;
  int32_t major = 0;
  if (valid) {
    const uint64_t k = key[s];
    major = (int32_t)(k >> bits_minor);
    minor_out[s] = (int32_t)(k & mmask);
    val_out[s] = val[s];
    is_head = (s == 0) || ((int32_t)(key[s - 1] >> bits_minor) != major);
    if (is_head) ptr[major] = (int32_t)s;
    if (s == nnz - 1) ptr[nrows] = (int32_t)nnz;
  }
  const uint64_t hb = __ballot(is_head);
  if ((threadIdx.x & 63) == 0 && valid) {
    head[s >> 6] = hb;
    tile_row[s >> 6] = major;
  }
}

// ------------------------------------------------------- CSR input

// rows[p] = lo + i for the entries p in [rowptr[i], rowptr[i+1]) (binary
// search per entry; a non-monotone rowptr only raises *err, every id stays in
// the range).
__global__ void k_csr_rows(int64_t n, const int64_t* __restrict__ rowptr, int64_t nnz, int64_t lo,
                           int64_t* __restrict__ rows) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = 0, b = n;   // largest i in [0, n) with rowptr[i] <= p
    while (b - a > 1) {
      const int64_t m = (a + b) >> 1;
      if (rowptr[m] <= p) a = m; else b = m;
    }
    rows[p] = lo + a;
  }
}

__global__ void k_csr_check(int64_t n, const int64_t* __restrict__ rowptr, int64_t nnz,
                            int32_t* __restrict__ err) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i <= n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = rowptr[i];
    if ((i == 0 && v != 0) || (i == n && v != nnz) || (i < n && rowptr[i + 1] < v) || v < 0 ||
        v > nnz)
      err[0] = 1;
  }
}

// ------------------------------------------- owner-grouped local order
//
// Method 2 of the paper's sparse communication model (SpC-SB / SpC-RB) stores
// local data as the concatenation of the data units exchanged with each peer,
// so that a message is sent or received in place.  With a group key per
// global id (for example 0 for the rows a processor owns and 1 + peer rank
// for the others), local ids are re-assigned in order of (key, global id):
// one stable radix pass over the used ids keyed by the group, whose values
// are the ids' offsets in the range, then the maps are rewritten.

// keys[l] = group of the l-th used id (in ascending id order), vals[l] = its
// offset in the range; a key outside [0, ngroups) raises *err.
__global__ void k_group_keys(int64_t n, const int64_t* __restrict__ gmap, int64_t lo,
                             const int32_t* __restrict__ group, int32_t ngroups,
                             uint64_t* __restrict__ keys, int32_t* __restrict__ vals,
                             int32_t* __restrict__ err) {
  for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < n;
       l += (int64_t)gridDim.x * blockDim.x) {
    const int64_t off = gmap[l] - lo;
    const int32_t k = group[off];
    const bool ok = k >= 0 && k < ngroups;
    if (!ok) err[0] = 1;
    keys[l] = ok ? (uint64_t)k : 0ull;
    vals[l] = (int32_t)off;
  }
}

// New local id j for the id at range offset sv[j].
__global__ void k_apply_order(int64_t n, const int32_t* __restrict__ sv, int64_t lo,
                              int64_t* __restrict__ gmap, int32_t* __restrict__ lmap) {
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const int32_t off = sv[j];
    gmap[j] = lo + off;
    lmap[off] = (int32_t)j;
  }
}

// goff[q] = number of used ids with key < q, for q = 0..ngroups (sorted keys).
__global__ void k_group_offsets(int32_t ngroups, int64_t n, const uint64_t* __restrict__ sk,
                                int32_t* __restrict__ goff) {
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q <= ngroups;
       q += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = 0, b = n;
    while (a < b) {
      const int64_t m = (a + b) >> 1;
      if (sk[m] < (uint64_t)q) a = m + 1; else b = m;
    }
    goff[q] = (int32_t)a;
  }
}

// gather (out[p] = in[perm[p]]) or scatter (out[perm[p]] = in[p]) of one
// value per entry; perm is the plan's slot -> caller map, or its column-major
// slot -> row-major slot map.
__global__ void k_permute(int64_t nnz, const int32_t* __restrict__ perm, int gather,
                          const float* __restrict__ in, float* __restrict__ out) {
  for (int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * blockDim.x) {
    if (gather)
      out[p] = in[perm[p]];
    else
      out[perm[p]] = in[p];
  }
}

// --------------------------------------------------------------- host side

namespace {

inline unsigned grid_for(int64_t n, int threads, int64_t cap = 1 << 20) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  if (b > cap) b = cap;
  return (unsigned)b;
}

struct Bump {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

struct Layout {
  size_t gmap_r, gmap_c, lmap_r, lmap_c, rowptr, colidx, perm, head, tile_row;
  size_t colptr, rowidx_t, slot_t, head_t, tile_col, small, goff_r, goff_c;
  size_t keys0, keys1, vals0, vals1, counts, partial;
  size_t total;
  int64_t sort_blocks, partial_len;
};

Layout make_layout(int64_t nnz, int64_t rr, int64_t cr, uint32_t flags) {
  Layout L{};
  Bump b;
  const int64_t cap_r = nnz < rr ? nnz : rr;
  const int64_t cap_c = nnz < cr ? nnz : cr;
  const int64_t ntiles = (nnz + 63) / 64;
  const bool csc = flags & SPC3D_BUILD_CSC;
  L.gmap_r = b.take(8 * (size_t)cap_r);
  L.gmap_c = b.take(8 * (size_t)cap_c);
  L.lmap_r = b.take(4 * (size_t)rr);
  L.lmap_c = b.take(4 * (size_t)cr);
  L.rowptr = b.take(4 * (size_t)(cap_r + 1));
  // colidx and perm are one region: before the slots are built it holds the
  // int64 row ids expanded from a CSR input (plan_create_csr)
  L.colidx = b.take(8 * (size_t)nnz);
  L.perm = L.colidx + 4 * (size_t)nnz;
  L.head = b.take(8 * (size_t)ntiles);
  L.tile_row = b.take(4 * (size_t)ntiles);
  L.colptr = csc ? b.take(4 * (size_t)(cap_c + 1)) : 0;
  L.rowidx_t = csc ? b.take(4 * (size_t)nnz) : 0;
  L.slot_t = csc ? b.take(4 * (size_t)nnz) : 0;
  L.head_t = csc ? b.take(8 * (size_t)ntiles) : 0;
  L.tile_col = csc ? b.take(4 * (size_t)ntiles) : 0;
  L.small = b.take(256);
  L.goff_r = b.take(4 * (size_t)(kMaxGroups + 1));
  L.goff_c = b.take(4 * (size_t)(kMaxGroups + 1));
  // temporaries (dead after plan creation)
  L.sort_blocks = (nnz + kSortTile - 1) / kSortTile;
  L.keys0 = b.take(8 * (size_t)nnz);
  L.keys1 = b.take(8 * (size_t)nnz);
  L.vals0 = b.take(4 * (size_t)nnz);
  L.vals1 = b.take(4 * (size_t)nnz);
  L.counts = b.take(4 * (size_t)(256 * L.sort_blocks));
  int64_t scan_max = rr > cr ? rr : cr;
  if (256 * L.sort_blocks > scan_max) scan_max = 256 * L.sort_blocks;
  L.partial_len = (scan_max + kScanTile - 1) / kScanTile + 1;
  L.partial = b.take(4 * (size_t)L.partial_len);
  L.total = b.off;
  return L;
}

spc3d_status scan_exclusive(int32_t* data, int64_t n, int32_t* partial, int32_t* total,
                            hipStream_t s) {
  if (n <= 0) return SPC3D_OK;
  const int64_t nb = (n + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n,
                     partial);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partial, nb, total);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(kScanThreads), 0, s, data, n,
                     partial, data);
  SPC3D_LAUNCHED("scan");
  return SPC3D_OK;
}

// Localize one axis: flags -> lmap, gmap; the count lands in *d_count.
spc3d_status localize(int64_t nnz, const int64_t* gid, int64_t lo, int64_t range, int32_t* lmap,
                      int64_t* gmap, int32_t* partial, int32_t* d_count, int32_t* d_err,
                      hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(range, 256)), dim3(256), 0, s, lmap, range, 0);
  if (nnz > 0)
    hipLaunchKernelGGL(k_mark, dim3(grid_for(nnz, 256)), dim3(256), 0, s, nnz, gid, lo,
                       lo + range, lmap, d_err);
  const int64_t nb = (range + kScanTile - 1) / kScanTile;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(kScanThreads), 0, s, lmap, range,
                     partial);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(1024), 0, s, partial, nb, d_count);
  hipLaunchKernelGGL(k_compact, dim3((unsigned)nb), dim3(kScanThreads), 0, s, lmap, range, lo,
                     partial, gmap);
  SPC3D_LAUNCHED("localize");
  return SPC3D_OK;
}

// Stable LSD sort of (key, val) over the low `bits` bits.  The result ends in
// (k0, v0) or (k1, v1); *out_k / *out_v point at it.
spc3d_status radix_sort(uint64_t* k0, int32_t* v0, uint64_t* k1, int32_t* v1, int64_t n,
                        int bits, int32_t* counts, int64_t nblk, int32_t* partial,
                        hipStream_t s, uint64_t** out_k, int32_t** out_v) {
  uint64_t* ks = k0;
  int32_t* vs = v0;
  uint64_t* kd = k1;
  int32_t* vd = v1;
  for (int shift = 0; shift < bits; shift += 8) {
    hipLaunchKernelGGL(k_radix_hist, dim3((unsigned)nblk), dim3(kSortThreads), 0, s, ks, n,
                       shift, nblk, counts);
    spc3d_status st = scan_exclusive(counts, 256 * nblk, partial, nullptr, s);
    if (st != SPC3D_OK) return st;
    hipLaunchKernelGGL(k_radix_scatter, dim3((unsigned)nblk), dim3(kSortThreads), 0, s, ks, vs,
                       n, shift, nblk, counts, kd, vd);
    SPC3D_LAUNCHED("radix pass");
    uint64_t* tk = ks; ks = kd; kd = tk;
    int32_t* tv = vs; vs = vd; vd = tv;
  }
  *out_k = ks;
  *out_v = vs;
  return SPC3D_OK;
}

// Re-assigns the local ids of one axis in (group, id) order (see above).
spc3d_status group_axis(int64_t n, int64_t lo, int64_t* gmap, int32_t* lmap,
                        const int32_t* group, int32_t ngroups, int32_t* goff, uint64_t* k0,
                        int32_t* v0, uint64_t* k1, int32_t* v1, int32_t* counts,
                        int32_t* partial, int32_t* d_err, hipStream_t s) {
  if (n > 0) {
    hipLaunchKernelGGL(k_group_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, n, gmap, lo, group,
                       ngroups, k0, v0, d_err);
    SPC3D_LAUNCHED("group keys");
    uint64_t* sk;
    int32_t* sv;
    const int64_t nblk = (n + kSortTile - 1) / kSortTile;
    spc3d_status st = radix_sort(k0, v0, k1, v1, n, ceil_log2(ngroups), counts, nblk, partial,
                                 s, &sk, &sv);
    if (st != SPC3D_OK) return st;
    hipLaunchKernelGGL(k_apply_order, dim3(grid_for(n, 256)), dim3(256), 0, s, n, sv, lo, gmap,
                       lmap);
    hipLaunchKernelGGL(k_group_offsets, dim3(grid_for(ngroups + 1, 256)), dim3(256), 0, s,
                       ngroups, n, sk, goff);
  } else {
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(ngroups + 1, 256)), dim3(256), 0, s, goff,
                       (int64_t)ngroups + 1, 0);
  }
  SPC3D_LAUNCHED("group order");
  return SPC3D_OK;
}

spc3d_status validate_ranges(int64_t nnz, int64_t row_lo, int64_t row_hi, int64_t col_lo,
                             int64_t col_hi) {
  if (nnz < 0 || nnz > INT32_MAX - 64)
    return fail(SPC3D_ERR_INVALID_ARG, "nnz=%lld outside [0, 2^31-65]", (long long)nnz);
  // hi > lo first, so the unsigned difference is the exact width of the range
  if (row_hi <= row_lo || (uint64_t)row_hi - (uint64_t)row_lo > (uint64_t)INT32_MAX - 1 ||
      col_hi <= col_lo || (uint64_t)col_hi - (uint64_t)col_lo > (uint64_t)INT32_MAX - 1)
    return fail(SPC3D_ERR_INVALID_ARG, "id ranges must hold 1..2^31-2 ids");
  return SPC3D_OK;
}

}  // namespace
}  // namespace spc3d

using namespace spc3d;

extern "C" {

spc3d_status spc3d_plan_workspace_size(int64_t nnz, int64_t row_lo, int64_t row_hi,
                                       int64_t col_lo, int64_t col_hi, uint32_t flags,
                                       size_t* bytes) {
  if (!bytes) return fail(SPC3D_ERR_INVALID_ARG, "bytes is NULL");
  spc3d_status st = validate_ranges(nnz, row_lo, row_hi, col_lo, col_hi);
  if (st != SPC3D_OK) return st;
  if (flags & ~uint32_t(SPC3D_BUILD_CSC)) return fail(SPC3D_ERR_INVALID_ARG, "unknown flags");
  *bytes = make_layout(nnz, row_hi - row_lo, col_hi - col_lo, flags).total;
  return SPC3D_OK;
}

}  // extern "C"

namespace {

spc3d_status create_plan(spc3d_plan* out, int64_t nnz, const int64_t* d_row_gid,
                         const int64_t* d_rowptr, const int64_t* d_col_gid, int64_t row_lo,
                         int64_t row_hi,
                         int64_t col_lo, int64_t col_hi, const int32_t* d_group_r,
                         int32_t ngroups_r, const int32_t* d_group_c, int32_t ngroups_c,
                         uint32_t flags, void* d_ws, size_t ws_bytes, hipStream_t stream) {
  if (!out) return fail(SPC3D_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  spc3d_status st = validate_ranges(nnz, row_lo, row_hi, col_lo, col_hi);
  if (st != SPC3D_OK) return st;
  if (flags & ~uint32_t(SPC3D_BUILD_CSC)) return fail(SPC3D_ERR_INVALID_ARG, "unknown flags");
  if (nnz > 0 && ((!d_row_gid && !d_rowptr) || !d_col_gid))
    return fail(SPC3D_ERR_INVALID_ARG, "id arrays are NULL");
  if (!d_ws) return fail(SPC3D_ERR_INVALID_ARG, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(d_ws) & 255u)
    return fail(SPC3D_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  const int64_t rr = row_hi - row_lo, cr = col_hi - col_lo;
  const Layout L = make_layout(nnz, rr, cr, flags);
  if (ws_bytes < L.total)
    return fail(SPC3D_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes, L.total);

  int device = 0;
  SPC3D_HIP(hipGetDevice(&device));
  char* w = static_cast<char*>(d_ws);
  Plan* p = new Plan();
  p->magic = kPlanMagic;
  p->device = device;
  p->flags = flags;
  p->nnz = nnz;
  p->row_lo = row_lo; p->row_hi = row_hi; p->col_lo = col_lo; p->col_hi = col_hi;
  p->ntiles = (nnz + 63) / 64;
  p->gmap_r = reinterpret_cast<int64_t*>(w + L.gmap_r);
  p->gmap_c = reinterpret_cast<int64_t*>(w + L.gmap_c);
  p->lmap_r = reinterpret_cast<int32_t*>(w + L.lmap_r);
  p->lmap_c = reinterpret_cast<int32_t*>(w + L.lmap_c);
  p->rowptr = reinterpret_cast<int32_t*>(w + L.rowptr);
  p->colidx = reinterpret_cast<int32_t*>(w + L.colidx);
  p->perm = reinterpret_cast<int32_t*>(w + L.perm);
  p->head = reinterpret_cast<uint64_t*>(w + L.head);
  p->tile_row = reinterpret_cast<int32_t*>(w + L.tile_row);
  if (flags & SPC3D_BUILD_CSC) {
    p->colptr = reinterpret_cast<int32_t*>(w + L.colptr);
    p->rowidx_t = reinterpret_cast<int32_t*>(w + L.rowidx_t);
    p->slot_t = reinterpret_cast<int32_t*>(w + L.slot_t);
    p->head_t = reinterpret_cast<uint64_t*>(w + L.head_t);
    p->tile_col = reinterpret_cast<int32_t*>(w + L.tile_col);
  }
  int32_t* small = reinterpret_cast<int32_t*>(w + L.small);
  uint64_t* keys0 = reinterpret_cast<uint64_t*>(w + L.keys0);
  uint64_t* keys1 = reinterpret_cast<uint64_t*>(w + L.keys1);
  int32_t* vals0 = reinterpret_cast<int32_t*>(w + L.vals0);
  int32_t* vals1 = reinterpret_cast<int32_t*>(w + L.vals1);
  int32_t* counts = reinterpret_cast<int32_t*>(w + L.counts);
  int32_t* partial = reinterpret_cast<int32_t*>(w + L.partial);
  if (d_group_r) {
    p->ngroups_r = ngroups_r;
    p->goff_r = reinterpret_cast<int32_t*>(w + L.goff_r);
  }
  if (d_group_c) {
    p->ngroups_c = ngroups_c;
    p->goff_c = reinterpret_cast<int32_t*>(w + L.goff_c);
  }

  auto bail = [&](spc3d_status s) {
    delete p;
    return s;
  };
  hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, small, (int64_t)64, 0);
  if (d_rowptr) {
    // CSR input: check the row pointer, expand it to one row id per entry in
    // the colidx / perm region (free until the slots are built)
    hipLaunchKernelGGL(k_csr_check, dim3(grid_for(rr + 1, 256)), dim3(256), 0, stream, rr,
                       d_rowptr, nnz, small + 4);
    if (nnz > 0) {
      int64_t* rows_tmp = reinterpret_cast<int64_t*>(w + L.colidx);
      hipLaunchKernelGGL(k_csr_rows, dim3(grid_for(nnz, 256)), dim3(256), 0, stream, rr, d_rowptr,
                         nnz, row_lo, rows_tmp);
      d_row_gid = rows_tmp;
    }
    SPC3D_LAUNCHED("csr rows");
  }
  st = localize(nnz, d_row_gid, row_lo, rr, p->lmap_r, p->gmap_r, partial, small + 0,
                small + 2, stream);
  if (st != SPC3D_OK) return bail(st);
  st = localize(nnz, d_col_gid, col_lo, cr, p->lmap_c, p->gmap_c, partial, small + 1,
                small + 2, stream);
  if (st != SPC3D_OK) return bail(st);
  int32_t host_small[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  hipError_t e = hipMemcpyAsync(host_small, small, sizeof host_small, hipMemcpyDeviceToHost,
                                stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return bail(hip_fail(e, "plan_create sync"));
  if (host_small[4])
    return bail(fail(SPC3D_ERR_INVALID_ARG,
                     "rowptr must start at 0, not decrease, and end at nnz"));
  if (host_small[2])
    return bail(fail(SPC3D_ERR_OUT_OF_RANGE, "a global id lies outside its [lo, hi) range"));
  p->R = host_small[0];
  p->C = host_small[1];
  if (d_group_r || d_group_c) {
    if (d_group_r) {
      st = group_axis(p->R, row_lo, p->gmap_r, p->lmap_r, d_group_r, ngroups_r, p->goff_r, keys0,
                      vals0, keys1, vals1, counts, partial, small + 3, stream);
      if (st != SPC3D_OK) return bail(st);
    }
    if (d_group_c) {
      st = group_axis(p->C, col_lo, p->gmap_c, p->lmap_c, d_group_c, ngroups_c, p->goff_c, keys0,
                      vals0, keys1, vals1, counts, partial, small + 3, stream);
      if (st != SPC3D_OK) return bail(st);
    }
    int32_t host_err = 0;
    e = hipMemcpyAsync(&host_err, small + 3, sizeof host_err, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
    if (e != hipSuccess) return bail(hip_fail(e, "plan_create group sync"));
    if (host_err) return bail(fail(SPC3D_ERR_INVALID_ARG, "a group key lies outside [0, ngroups)"));
  }

  const int bits_r = ceil_log2(p->R), bits_c = ceil_log2(p->C);
  if (nnz > 0) {
    hipLaunchKernelGGL(k_make_keys, dim3(grid_for(nnz, 256)), dim3(256), 0, stream, nnz,
                       d_row_gid, d_col_gid, row_lo, col_lo, p->lmap_r, p->lmap_c, bits_c, keys0,
                       vals0);
    SPC3D_LAUNCHED("make_keys");
    uint64_t* sk;
    int32_t* sv;
    st = radix_sort(keys0, vals0, keys1, vals1, nnz, bits_r + bits_c, counts, L.sort_blocks,
                    partial, stream, &sk, &sv);
    if (st != SPC3D_OK) return bail(st);
    hipLaunchKernelGGL(k_build_slots, dim3(grid_for(nnz, 256, INT32_MAX)), dim3(256), 0, stream,
                       nnz, p->R, sk, sv, bits_c, p->colidx, p->perm, p->rowptr, p->head,
                       p->tile_row);
    SPC3D_LAUNCHED("build_slots");
    if (flags & SPC3D_BUILD_CSC) {
      uint64_t* tk = (sk == keys0) ? keys1 : keys0;
      int32_t* tv = (sv == vals0) ? vals1 : vals0;
      hipLaunchKernelGGL(k_make_keys_t, dim3(grid_for(nnz, 256)), dim3(256), 0, stream, nnz, sk,
                         bits_c, bits_r, tk, tv);
      SPC3D_LAUNCHED("make_keys_t");
      uint64_t* ok = (tk == keys0) ? keys1 : keys0;
      int32_t* ov = (tv == vals0) ? vals1 : vals0;
      uint64_t* sk2;
      int32_t* sv2;
      st = radix_sort(tk, tv, ok, ov, nnz, bits_r + bits_c, counts, L.sort_blocks, partial,
                      stream, &sk2, &sv2);
      if (st != SPC3D_OK) return bail(st);
      hipLaunchKernelGGL(k_build_slots, dim3(grid_for(nnz, 256, INT32_MAX)), dim3(256), 0,
                         stream, nnz, p->C, sk2, sv2, bits_r, p->rowidx_t, p->slot_t, p->colptr,
                         p->head_t, p->tile_col);
      SPC3D_LAUNCHED("build_slots_t");
    }
  } else {
    hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, p->rowptr, (int64_t)1, 0);
    if (flags & SPC3D_BUILD_CSC)
      hipLaunchKernelGGL(k_fill_i32, dim3(1), dim3(64), 0, stream, p->colptr, (int64_t)1, 0);
    SPC3D_LAUNCHED("empty plan");
  }
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return bail(hip_fail(e, "plan_create final sync"));
  {
    std::lock_guard<std::mutex> lk(g_plans_mu);
    g_plans.insert(static_cast<const void*>(p));
  }
  *out = reinterpret_cast<spc3d_plan>(p);
  return SPC3D_OK;
}

}  // namespace

extern "C" {

spc3d_status spc3d_plan_create_coo(spc3d_plan* out, int64_t nnz, const int64_t* d_row_gid,
                                   const int64_t* d_col_gid, int64_t row_lo, int64_t row_hi,
                                   int64_t col_lo, int64_t col_hi, uint32_t flags, void* d_ws,
                                   size_t ws_bytes, hipStream_t stream) {
  return create_plan(out, nnz, d_row_gid, nullptr, d_col_gid, row_lo, row_hi, col_lo, col_hi,
                     nullptr, 0, nullptr, 0, flags, d_ws, ws_bytes, stream);
}

spc3d_status spc3d_plan_create_csr(spc3d_plan* out, int64_t nnz, const int64_t* d_rowptr,
                                   const int64_t* d_col_gid, int64_t row_lo, int64_t row_hi,
                                   int64_t col_lo, int64_t col_hi, uint32_t flags, void* d_ws,
                                   size_t ws_bytes, hipStream_t stream) {
  if (out) *out = nullptr;
  if (!d_rowptr) return fail(SPC3D_ERR_INVALID_ARG, "rowptr is NULL");
  return create_plan(out, nnz, nullptr, d_rowptr, d_col_gid, row_lo, row_hi, col_lo, col_hi,
                     nullptr, 0, nullptr, 0, flags, d_ws, ws_bytes, stream);
}

spc3d_status spc3d_plan_create_coo_grouped(spc3d_plan* out, int64_t nnz,
                                           const int64_t* d_row_gid, const int64_t* d_col_gid,
                                           int64_t row_lo, int64_t row_hi, int64_t col_lo,
                                           int64_t col_hi, const int32_t* d_group_r,
                                           int32_t ngroups_r, const int32_t* d_group_c,
                                           int32_t ngroups_c, uint32_t flags, void* d_ws,
                                           size_t ws_bytes, hipStream_t stream) {
  if (out) *out = nullptr;
  if ((d_group_r && (ngroups_r < 1 || ngroups_r > kMaxGroups)) ||
      (d_group_c && (ngroups_c < 1 || ngroups_c > kMaxGroups)))
    return fail(SPC3D_ERR_INVALID_ARG, "ngroups must lie in [1, %d]", kMaxGroups);
  return create_plan(out, nnz, d_row_gid, nullptr, d_col_gid, row_lo, row_hi, col_lo, col_hi,
                     d_group_r, ngroups_r, d_group_c, ngroups_c, flags, d_ws, ws_bytes, stream);
}

spc3d_status spc3d_plan_group_offsets(spc3d_plan h, spc3d_axis axis, const int32_t** d_offsets,
                                      int32_t* ngroups) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (axis != SPC3D_ROWS && axis != SPC3D_COLS) return fail(SPC3D_ERR_INVALID_ARG, "bad axis");
  const int32_t* g = axis == SPC3D_ROWS ? p->goff_r : p->goff_c;
  if (!g) return fail(SPC3D_ERR_INVALID_ARG, "the plan was built without groups on this axis");
  if (d_offsets) *d_offsets = g;
  if (ngroups) *ngroups = axis == SPC3D_ROWS ? p->ngroups_r : p->ngroups_c;
  return SPC3D_OK;
}

spc3d_status spc3d_plan_query(spc3d_plan h, int64_t* R, int64_t* C, int64_t* nnz) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (R) *R = p->R;
  if (C) *C = p->C;
  if (nnz) *nnz = p->nnz;
  return SPC3D_OK;
}

spc3d_status spc3d_plan_maps(spc3d_plan h, spc3d_maps* m) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (!m) return fail(SPC3D_ERR_INVALID_ARG, "maps is NULL");
  m->gmap_r = p->gmap_r; m->gmap_c = p->gmap_c;
  m->lmap_r = p->lmap_r; m->lmap_c = p->lmap_c;
  m->rowptr = p->rowptr; m->colidx = p->colidx; m->perm = p->perm;
  m->colptr = p->colptr; m->rowidx_t = p->rowidx_t; m->slot_t = p->slot_t;
  return SPC3D_OK;
}

spc3d_status spc3d_plan_destroy(spc3d_plan h) {
  std::lock_guard<std::mutex> lk(g_plans_mu);
  if (!h || !g_plans.erase(static_cast<const void*>(h)))
    return fail(SPC3D_ERR_BAD_HANDLE, "not a live plan");
  Plan* p = reinterpret_cast<Plan*>(h);
  p->magic = 0;
  delete p;
  return SPC3D_OK;
}

spc3d_status spc3d_permute_values(spc3d_plan h, int direction, const float* d_in, float* d_out,
                                  hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (direction < SPC3D_CALLER_TO_SLOT || direction > SPC3D_COLUMN_TO_SLOT)
    return fail(SPC3D_ERR_INVALID_ARG, "bad direction %d", direction);
  const bool csc = direction == SPC3D_SLOT_TO_COLUMN || direction == SPC3D_COLUMN_TO_SLOT;
  if (csc && !(p->flags & SPC3D_BUILD_CSC))
    return fail(SPC3D_ERR_INVALID_ARG, "column-major order needs a plan built with BUILD_CSC");
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_in || !d_out) return fail(SPC3D_ERR_INVALID_ARG, "NULL array");
  if (d_in == d_out) return fail(SPC3D_ERR_INVALID_ARG, "in and out alias");
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
  const int gather = direction == SPC3D_CALLER_TO_SLOT || direction == SPC3D_SLOT_TO_COLUMN;
  hipLaunchKernelGGL(k_permute, dim3(grid_for(p->nnz, 256)), dim3(256), 0, stream, p->nnz,
                     csc ? p->slot_t : p->perm, gather, d_in, d_out);
  SPC3D_LAUNCHED("permute_values");
  return SPC3D_OK;
}

const char* spc3d_status_string(spc3d_status s) {
  switch (s) {
    case SPC3D_OK: return "ok";
    case SPC3D_ERR_INVALID_ARG: return "invalid argument";
    case SPC3D_ERR_OUT_OF_RANGE: return "global id out of range";
    case SPC3D_ERR_WORKSPACE: return "workspace or buffer too small";
    case SPC3D_ERR_UNSUPPORTED: return "unsupported";
    case SPC3D_ERR_HIP: return "HIP runtime error";
    case SPC3D_ERR_BAD_HANDLE: return "bad plan handle";
  }
  return "unknown status";
}

const char* spc3d_last_error(void) { return g_last_error.c_str(); }

int spc3d_version(void) { return 100; }

}  // extern "C"
