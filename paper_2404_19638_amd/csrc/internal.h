// Internal declarations shared by the spc3d HIP sources (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>

#include "../../include/spc3d.h"

namespace spc3d {

constexpr uint64_t kPlanMagic = 0x53504333444c4f43ull;
constexpr int kMaxKz = 1024;
constexpr int kMaxKzScalar = 256;
constexpr int kMaxGroups = 4096;   // owner groups per axis of a grouped plan

// One orientation of the localized block: row-major (CSR) or column-major.
// Slots are grouped into 64-slot tiles; head[t] bit i is set when slot
// 64*t + i starts a row, tile_row[t] is the row of slot 64*t.
struct Orient {
  int64_t nnz = 0;
  int64_t nrows = 0;        // rows of this orientation (R for CSR, C for CSC)
  int64_t ncols = 0;
  const int32_t* ptr = nullptr;
  const int32_t* idx = nullptr;
  const uint64_t* head = nullptr;
  const int32_t* tile_row = nullptr;
  const int32_t* vidx = nullptr;   // slot of the value array (CSC: row-major slot)
};

struct Plan {
  uint64_t magic = 0;
  int device = 0;
  uint32_t flags = 0;
  int64_t nnz = 0, R = 0, C = 0;
  int64_t row_lo = 0, row_hi = 0, col_lo = 0, col_hi = 0;
  int64_t ntiles = 0;
  int64_t* gmap_r = nullptr;
  int64_t* gmap_c = nullptr;
  int32_t* lmap_r = nullptr;
  int32_t* lmap_c = nullptr;
  int32_t* rowptr = nullptr;
  int32_t* colidx = nullptr;
  int32_t* perm = nullptr;
  uint64_t* head = nullptr;
  int32_t* tile_row = nullptr;
  int32_t* colptr = nullptr;
  int32_t* rowidx_t = nullptr;
  int32_t* slot_t = nullptr;
  uint64_t* head_t = nullptr;
  int32_t* tile_col = nullptr;
  int32_t ngroups_r = 0, ngroups_c = 0;   // owner-grouped local order (0: ascending ids)
  int32_t* goff_r = nullptr;              // [ngroups + 1] first local id of each group
  int32_t* goff_c = nullptr;

  Orient csr() const {
    Orient o;
    o.nnz = nnz; o.nrows = R; o.ncols = C;
    o.ptr = rowptr; o.idx = colidx; o.head = head; o.tile_row = tile_row; o.vidx = nullptr;
    return o;
  }
  Orient csc() const {
    Orient o;
    o.nnz = nnz; o.nrows = C; o.ncols = R;
    o.ptr = colptr; o.idx = rowidx_t; o.head = head_t; o.tile_row = tile_col; o.vidx = slot_t;
    return o;
  }
};

// Error reporting: records a thread-local message and returns the status.
spc3d_status fail(spc3d_status s, const char* fmt, ...);
spc3d_status hip_fail(hipError_t e, const char* what);
// Resolves a handle to a live plan (BAD_HANDLE otherwise).
spc3d_status get_plan(spc3d_plan h, Plan** out);
// Makes the plan's device current for the calling thread until the guard
// goes out of scope, then gives the thread back the device it had.
class DeviceGuard {
 public:
  DeviceGuard() = default;
  DeviceGuard(const DeviceGuard&) = delete;
  DeviceGuard& operator=(const DeviceGuard&) = delete;
  spc3d_status enter(const Plan* p);
  ~DeviceGuard() {
    if (prev_ >= 0) (void)hipSetDevice(prev_);
  }

 private:
  int prev_ = -1;   // the caller's device when enter() switched away from it
};

#define SPC3D_HIP(call)                                  \
  do {                                                   \
    hipError_t e_ = (call);                              \
    if (e_ != hipSuccess) return ::spc3d::hip_fail(e_, #call); \
  } while (0)

// Checks the plan's local ids on the device (spc3d_plan_check); synchronizes
// the stream.
spc3d_status check_plan(Plan* p, hipStream_t stream);
// check_plan when SPC3D_DEBUG_BOUNDS is set (to anything but "0") in the
// environment, read once per process; SPC3D_OK otherwise.
spc3d_status debug_check(Plan* p, hipStream_t stream);
#define SPC3D_DEBUG_CHECK(plan, stream)                                   \
  do {                                                                    \
    spc3d_status d_ = ::spc3d::debug_check((plan), (stream));             \
    if (d_ != SPC3D_OK) return d_;                                        \
  } while (0)

#define SPC3D_LAUNCHED(what)                                     \
  do {                                                           \
    hipError_t e_ = hipGetLastError();                           \
    if (e_ != hipSuccess) return ::spc3d::hip_fail(e_, what);    \
  } while (0)

inline bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

inline int ceil_log2(int64_t n) {
  int b = 0;
  while (b < 62 && (int64_t(1) << b) < n) ++b;
  return b;
}

// Kernel-variant decoding shared by SDDMM and SpMM.
struct Variant {
  int lanes;   // lanes per nonzero (2..64)
  int items;   // slots per wavefront work item (64..1024)
};

// Work items are mapped to workgroups so that each of the 8 XCDs (which
// receive workgroups round-robin) processes one contiguous range of items:
// neighbouring items share dense rows through the same L2.
__device__ inline int64_t xcd_block(int64_t nblocks) {
  const int64_t b = blockIdx.x;
  const int64_t x = b & 7, i = b >> 3;
  const int64_t q = nblocks >> 3, r = nblocks & 7;
  return x * q + (x < r ? x : r) + i;
}

__device__ inline uint64_t lanemask_le(int lane) {
  return lane >= 63 ? ~0ull : ((2ull << lane) - 1ull);
}

}  // namespace spc3d
