// Sparsity-aware communication accounting of a Dist3D distribution (paper:
// Section "Sparsity-aware Communication Analysis of 3D SDDMM" and Algorithm 1,
// "Parallel lambda-aware random distribution", in Section "The SpComm3D
// Framework").
//
// For one row block x of the X x Y grid (or, with the roles swapped, one
// column block), the Y processors P_{x,y,:} hold the blocks S_{x,y}; part y
// uses the dense rows of the distinct row ids of S_{x,y} (its globalMap, the
// gmap_r of its localized plan).  For every id i of the block's range:
//
//   lambda_i = number of parts whose block has a nonzero in row i;
//   owner_i  = one of those parts, chosen uniformly at random (Algorithm 1:
//              the candidates of a row are exactly the parts that use it, so
//              the owner is always one of them and no row travels to a
//              processor that does not need it);
//   owned_p  = number of ids part p owns;
//   comm[p][q] = number of ids part p uses and part q owns (q != p): the rows
//              p receives from q in the PreComm phase (the communication
//              graph of the paper's Eq. for commG), so part p receives
//              R_p - owned_p rows in all and the total is sum_i (lambda_i - 1).
//
// The random pick takes one 64-bit draw r_i per id (passed in) and the
// candidate of rank floor(r_i * lambda_i / 2^64) in ascending part order.
// All outputs are integers and independent of scheduling (atomic integer
// additions commute).  Up to 64 parts per block row (a 64-bit candidate mask
// per id).
#include "internal.h"

namespace spc3d {

__global__ void k_fill_u64(int64_t n, uint64_t* __restrict__ a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

__global__ void k_fill_i64(int64_t n, int64_t* __restrict__ a) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    a[i] = 0;
}

// Marks part p as a candidate of every id in its globalMap (ids outside the
// range are skipped; the host reports them).
__global__ void k_mark_part(int64_t n, const int64_t* __restrict__ gmap, int64_t lo, int64_t range,
                            int part, unsigned long long* __restrict__ mask,
                            unsigned long long* __restrict__ bad) {
  for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < n;
       l += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = gmap[l] - lo;
    if (g >= 0 && g < range)
      atomicOr(mask + g, 1ull << part);
    else
      atomicAdd(bad, 1ull);
  }
}

__global__ void k_pick_owner(int64_t n, const unsigned long long* __restrict__ mask,
                             const uint64_t* __restrict__ rnd, int32_t* __restrict__ lambda,
                             int32_t* __restrict__ owner,
                             unsigned long long* __restrict__ owned) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    unsigned long long m = mask[i];
    const int lam = __popcll(m);
    int o = -1;
    if (lam > 0) {
      const int k = rnd ? (int)__umul64hi(rnd[i], (unsigned long long)lam) : 0;
      for (int j = 0; j < k; ++j) m &= m - 1ull;   // drop the k lowest candidates
      o = __ffsll((long long)m) - 1;
      atomicAdd(owned + o, 1ull);
    }
    lambda[i] = lam;
    owner[i] = o;
  }
}

// comm[part * nparts + q] += 1 for every id of part whose owner q != part.
__global__ void k_count_comm(int64_t n, const int64_t* __restrict__ gmap, int64_t lo,
                             int64_t range, int part, int nparts,
                             const int32_t* __restrict__ owner,
                             unsigned long long* __restrict__ comm) {
  for (int64_t l = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; l < n;
       l += (int64_t)gridDim.x * blockDim.x) {
    const int64_t g = gmap[l] - lo;
    if (g < 0 || g >= range) continue;
    const int q = owner[g];
    if (q != part) atomicAdd(comm + (int64_t)part * nparts + q, 1ull);
  }
}

namespace {

unsigned grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 65536) b = 65536;
  return (unsigned)b;
}

}  // namespace
}  // namespace spc3d

using namespace spc3d;

extern "C" {

spc3d_status spc3d_lambda_owners_workspace_size(int64_t lo, int64_t hi, size_t* bytes) {
  if (!bytes) return fail(SPC3D_ERR_INVALID_ARG, "bytes is NULL");
  if (hi <= lo) return fail(SPC3D_ERR_INVALID_ARG, "empty id range [%lld, %lld)", (long long)lo,
                            (long long)hi);
  *bytes = (size_t)(hi - lo) * 8 + 256;   // candidate masks, then an error counter
  return SPC3D_OK;
}

spc3d_status spc3d_lambda_owners(int32_t nparts, const int64_t* const* h_gmaps,
                                 const int64_t* h_counts, int64_t lo, int64_t hi,
                                 const uint64_t* d_rand, int32_t* d_lambda, int32_t* d_owner,
                                 int64_t* d_owned, int64_t* d_comm, void* d_ws, size_t ws_bytes,
                                 hipStream_t stream) {
  if (nparts < 1 || nparts > 64) return fail(SPC3D_ERR_UNSUPPORTED, "nparts=%d outside [1,64]", nparts);
  if (!h_gmaps || !h_counts) return fail(SPC3D_ERR_INVALID_ARG, "NULL part arrays");
  if (hi <= lo) return fail(SPC3D_ERR_INVALID_ARG, "empty id range");
  const int64_t n = hi - lo;
  if (!d_lambda || !d_owner || !d_owned || !d_comm || !d_ws)
    return fail(SPC3D_ERR_INVALID_ARG, "NULL output or workspace");
  if (ws_bytes < (size_t)n * 8 + 256)
    return fail(SPC3D_ERR_WORKSPACE, "workspace %zu bytes < %zu required", ws_bytes,
                (size_t)n * 8 + 256);
  if (reinterpret_cast<uintptr_t>(d_ws) & 7u)
    return fail(SPC3D_ERR_INVALID_ARG, "workspace must be 8-byte aligned");
  for (int p = 0; p < nparts; ++p) {
    if (h_counts[p] < 0 || h_counts[p] > n)
      return fail(SPC3D_ERR_INVALID_ARG, "part %d has %lld ids for a range of %lld", p,
                  (long long)h_counts[p], (long long)n);
    if (h_counts[p] > 0 && !h_gmaps[p]) return fail(SPC3D_ERR_INVALID_ARG, "part %d: NULL gmap", p);
  }
  unsigned long long* mask = static_cast<unsigned long long*>(d_ws);
  unsigned long long* bad = mask + n;
  hipLaunchKernelGGL(k_fill_u64, dim3(grid_for(n + 1)), dim3(256), 0, stream, n + 1,
                     reinterpret_cast<uint64_t*>(mask));
  hipLaunchKernelGGL(k_fill_i64, dim3(1), dim3(256), 0, stream, (int64_t)nparts, d_owned);
  hipLaunchKernelGGL(k_fill_i64, dim3(grid_for((int64_t)nparts * nparts)), dim3(256), 0, stream,
                     (int64_t)nparts * nparts, d_comm);
  for (int p = 0; p < nparts; ++p)
    if (h_counts[p] > 0)
      hipLaunchKernelGGL(k_mark_part, dim3(grid_for(h_counts[p])), dim3(256), 0, stream,
                         h_counts[p], h_gmaps[p], lo, n, p, mask, bad);
  hipLaunchKernelGGL(k_pick_owner, dim3(grid_for(n)), dim3(256), 0, stream, n, mask, d_rand,
                     d_lambda, d_owner, reinterpret_cast<unsigned long long*>(d_owned));
  for (int p = 0; p < nparts; ++p)
    if (h_counts[p] > 0)
      hipLaunchKernelGGL(k_count_comm, dim3(grid_for(h_counts[p])), dim3(256), 0, stream,
                         h_counts[p], h_gmaps[p], lo, n, p, (int)nparts, d_owner,
                         reinterpret_cast<unsigned long long*>(d_comm));
  SPC3D_LAUNCHED("lambda_owners");
  // setup-time call: report ids outside [lo, hi) (synchronizes the stream)
  unsigned long long nbad = 0;
  SPC3D_HIP(hipMemcpyAsync(&nbad, bad, sizeof(nbad), hipMemcpyDeviceToHost, stream));
  SPC3D_HIP(hipStreamSynchronize(stream));
  if (nbad)
    return fail(SPC3D_ERR_OUT_OF_RANGE, "%llu ids of the parts lie outside [%lld, %lld)", nbad,
                (long long)lo, (long long)hi);
  return SPC3D_OK;
}

}  // extern "C"
