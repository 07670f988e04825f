// PreComm / PostComm, local side: SpC-BB packing and unpacking of data units
// (paper: Section "Sparse communication model", Method 1 — copy each global
// id's data unit into a buffer; at the receiver, put each one back at the
// location of its global id).  Here a data unit is the K-slice [k0, k0+kz) of
// one dense row, the packed buffer holds the units of the block's non-empty
// rows (or columns) in local-id order, and unpacking reduces (+=) into the
// owner's rows as the SpMM PostComm does ("Building SpMM with SpComm3D").
//
// Both kernels stream: every thread moves one 16-byte chunk (4 FP32 or 8
// bfloat16 values), so a packed FP32 row with kz = 32 is one 128-byte line.
#include "internal.h"
#include "vec.h"

namespace spc3d {

// packed[l*kz + k] = conv(src[(gmap[l]-lo)*ld + k0 + k]); VO output elements
// per thread.
template <typename Tin, typename Tout, int VO>
__global__ __launch_bounds__(256) void k_gather(int64_t n, const int64_t* __restrict__ gmap,
                                                int64_t lo, const Tin* __restrict__ src,
                                                int64_t ld, int k0, int kz,
                                                Tout* __restrict__ dst) {
  const int chunks = kz / VO;
  const int64_t total = n * chunks;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i / chunks;
    const int c = (int)(i - l * chunks);
    const Tin* s = src + (gmap[l] - lo) * ld + k0 + (int64_t)c * VO;
    Tout* d = dst + l * kz + (int64_t)c * VO;
    if constexpr (VO == 4 && sizeof(Tin) == 4 && sizeof(Tout) == 4) {
      *reinterpret_cast<float4*>(d) = *reinterpret_cast<const float4*>(s);
    } else if constexpr (VO == 8 && sizeof(Tin) == 4 && sizeof(Tout) == 2) {
      const float4 a = reinterpret_cast<const float4*>(s)[0];
      const float4 b = reinterpret_cast<const float4*>(s)[1];
      uint4 o;
      o.x = (uint32_t)f32_to_bf16(a.x) | ((uint32_t)f32_to_bf16(a.y) << 16);
      o.y = (uint32_t)f32_to_bf16(a.z) | ((uint32_t)f32_to_bf16(a.w) << 16);
      o.z = (uint32_t)f32_to_bf16(b.x) | ((uint32_t)f32_to_bf16(b.y) << 16);
      o.w = (uint32_t)f32_to_bf16(b.z) | ((uint32_t)f32_to_bf16(b.w) << 16);
      *reinterpret_cast<uint4*>(d) = o;
    } else if constexpr (VO == 8 && sizeof(Tin) == 2 && sizeof(Tout) == 2) {
      *reinterpret_cast<uint4*>(d) = *reinterpret_cast<const uint4*>(s);
    } else if constexpr (sizeof(Tin) == 4 && sizeof(Tout) == 2) {
      d[0] = f32_to_bf16(reinterpret_cast<const float*>(s)[0]);
    } else {
      d[0] = s[0];
    }
  }
}

// dst[(gmap[l]-lo)*ld + k0 + k] += packed[l*kz + k]; VO elements per thread.
template <int VO>
__global__ __launch_bounds__(256) void k_scatter_add(int64_t n, const int64_t* __restrict__ gmap,
                                                     int64_t lo, const float* __restrict__ packed,
                                                     int kz, float* __restrict__ dst, int64_t ld,
                                                     int k0) {
  const int chunks = kz / VO;
  const int64_t total = n * chunks;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t l = i / chunks;
    const int c = (int)(i - l * chunks);
    float* d = dst + (gmap[l] - lo) * ld + k0 + (int64_t)c * VO;
    const float* s = packed + l * kz + (int64_t)c * VO;
    if constexpr (VO == 4) {
      float4 a = *reinterpret_cast<const float4*>(d);
      const float4 b = *reinterpret_cast<const float4*>(s);
      a.x = a.x + b.x; a.y = a.y + b.y; a.z = a.z + b.z; a.w = a.w + b.w;
      *reinterpret_cast<float4*>(d) = a;
    } else {
      d[0] = d[0] + s[0];
    }
  }
}

static unsigned grid_chunks(int64_t total) {
  int64_t b = (total + 255) / 256;
  if (b < 1) b = 1;
  if (b > (1 << 20)) b = 1 << 20;
  return (unsigned)b;
}

}  // namespace spc3d

using namespace spc3d;

extern "C" {

spc3d_status spc3d_gather(spc3d_plan h, spc3d_axis axis, const void* d_src, spc3d_dtype src_t,
                          int64_t ld_src, int32_t k0, int32_t kz, void* d_packed,
                          spc3d_dtype packed_t, hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (axis != SPC3D_ROWS && axis != SPC3D_COLS) return fail(SPC3D_ERR_INVALID_ARG, "bad axis");
  if (src_t != SPC3D_F32 && src_t != SPC3D_BF16) return fail(SPC3D_ERR_INVALID_ARG, "bad src_t");
  if (packed_t != SPC3D_F32 && packed_t != SPC3D_BF16)
    return fail(SPC3D_ERR_INVALID_ARG, "bad packed_t");
  if (src_t == SPC3D_BF16 && packed_t == SPC3D_F32)
    return fail(SPC3D_ERR_UNSUPPORTED, "bfloat16 source to FP32 packing");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "kz=%d outside [1,%d]", kz, kMaxKz);
  if (k0 < 0 || ld_src < (int64_t)k0 + kz)
    return fail(SPC3D_ERR_INVALID_ARG, "k0=%d kz=%d do not fit ld_src=%lld", k0, kz,
                (long long)ld_src);
  const int64_t n = axis == SPC3D_ROWS ? p->R : p->C;
  if (n == 0) return SPC3D_OK;
  if (!d_src || !d_packed) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  st = use_device(p);
  if (st != SPC3D_OK) return st;
  const int64_t* gmap = axis == SPC3D_ROWS ? p->gmap_r : p->gmap_c;
  const int64_t lo = axis == SPC3D_ROWS ? p->row_lo : p->col_lo;
  const bool src_al = aligned16(d_src) && aligned16(d_packed);
  if (src_t == SPC3D_F32 && packed_t == SPC3D_F32) {
    const float* s = static_cast<const float*>(d_src);
    float* d = static_cast<float*>(d_packed);
    if (src_al && kz % 4 == 0 && ld_src % 4 == 0 && k0 % 4 == 0)
      hipLaunchKernelGGL((k_gather<float, float, 4>), dim3(grid_chunks(n * kz / 4)), dim3(256), 0,
                         stream, n, gmap, lo, s, ld_src, k0, kz, d);
    else
      hipLaunchKernelGGL((k_gather<float, float, 1>), dim3(grid_chunks(n * kz)), dim3(256), 0,
                         stream, n, gmap, lo, s, ld_src, k0, kz, d);
  } else if (src_t == SPC3D_F32) {
    const float* s = static_cast<const float*>(d_src);
    bf16_t* d = static_cast<bf16_t*>(d_packed);
    if (src_al && kz % 8 == 0 && ld_src % 4 == 0 && k0 % 4 == 0)
      hipLaunchKernelGGL((k_gather<float, bf16_t, 8>), dim3(grid_chunks(n * kz / 8)), dim3(256),
                         0, stream, n, gmap, lo, s, ld_src, k0, kz, d);
    else
      hipLaunchKernelGGL((k_gather<float, bf16_t, 1>), dim3(grid_chunks(n * kz)), dim3(256), 0,
                         stream, n, gmap, lo, s, ld_src, k0, kz, d);
  } else {
    const bf16_t* s = static_cast<const bf16_t*>(d_src);
    bf16_t* d = static_cast<bf16_t*>(d_packed);
    if (src_al && kz % 8 == 0 && ld_src % 8 == 0 && k0 % 8 == 0)
      hipLaunchKernelGGL((k_gather<bf16_t, bf16_t, 8>), dim3(grid_chunks(n * kz / 8)), dim3(256),
                         0, stream, n, gmap, lo, s, ld_src, k0, kz, d);
    else
      hipLaunchKernelGGL((k_gather<bf16_t, bf16_t, 1>), dim3(grid_chunks(n * kz)), dim3(256), 0,
                         stream, n, gmap, lo, s, ld_src, k0, kz, d);
  }
  SPC3D_LAUNCHED("gather");
  return SPC3D_OK;
}

spc3d_status spc3d_scatter_reduce(spc3d_plan h, spc3d_axis axis, const float* d_packed,
                                  int32_t kz, float* d_dst, int64_t ld_dst, int32_t k0,
                                  hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (axis != SPC3D_ROWS && axis != SPC3D_COLS) return fail(SPC3D_ERR_INVALID_ARG, "bad axis");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "kz=%d outside [1,%d]", kz, kMaxKz);
  if (k0 < 0 || ld_dst < (int64_t)k0 + kz)
    return fail(SPC3D_ERR_INVALID_ARG, "k0=%d kz=%d do not fit ld_dst=%lld", k0, kz,
                (long long)ld_dst);
  const int64_t n = axis == SPC3D_ROWS ? p->R : p->C;
  if (n == 0) return SPC3D_OK;
  if (!d_packed || !d_dst) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  st = use_device(p);
  if (st != SPC3D_OK) return st;
  const int64_t* gmap = axis == SPC3D_ROWS ? p->gmap_r : p->gmap_c;
  const int64_t lo = axis == SPC3D_ROWS ? p->row_lo : p->col_lo;
  if (aligned16(d_packed) && aligned16(d_dst) && kz % 4 == 0 && ld_dst % 4 == 0 && k0 % 4 == 0)
    hipLaunchKernelGGL(k_scatter_add<4>, dim3(grid_chunks(n * kz / 4)), dim3(256), 0, stream, n,
                       gmap, lo, d_packed, kz, d_dst, ld_dst, k0);
  else
    hipLaunchKernelGGL(k_scatter_add<1>, dim3(grid_chunks(n * kz)), dim3(256), 0, stream, n,
                       gmap, lo, d_packed, kz, d_dst, ld_dst, k0);
  SPC3D_LAUNCHED("scatter_reduce");
  return SPC3D_OK;
}

}  // extern "C"
