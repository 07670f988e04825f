// PreComm / PostComm, local side: SpC-BB packing and unpacking of data units
// (paper: Section "Sparse communication model", Method 1 — copy each global
// id's data unit into a buffer; at the receiver, put each one back at the
// location of its global id).  Here a data unit is the K-slice [k0, k0+kz) of
// one dense row, the packed buffer holds the units of the block's non-empty
// rows (or columns) in local-id order, and unpacking reduces (+=) into the
// owner's rows as the SpMM PostComm does ("Building SpMM with SpComm3D").
//
// Both kernels stream in 16-byte chunks (4 FP32 or 8 bfloat16 values), so a
// packed FP32 row with kz = 32 is one 128-byte line.
#include <type_traits>

#include "internal.h"
#include "vec.h"

namespace spc3d {

// Each thread moves kUnroll chunks of VO output elements, all loads of a
// thread issued before its stores (1 measured best: more threads in flight).
constexpr int kUnroll = 1;

template <typename Tin, typename Tout, int VO>
struct Chunk;

template <>
struct Chunk<float, float, 4> {
  float4 v;
  __device__ void load(const float* s) { v = *reinterpret_cast<const float4*>(s); }
  __device__ void store(float* d) const { *reinterpret_cast<float4*>(d) = v; }
};

template <>
struct Chunk<float, bf16_t, 8> {
  float4 a, b;
  __device__ void load(const float* s) {
    a = reinterpret_cast<const float4*>(s)[0];
    b = reinterpret_cast<const float4*>(s)[1];
  }
  __device__ void store(bf16_t* d) const {
    uint4 o;
    o.x = (uint32_t)f32_to_bf16(a.x) | ((uint32_t)f32_to_bf16(a.y) << 16);
    o.y = (uint32_t)f32_to_bf16(a.z) | ((uint32_t)f32_to_bf16(a.w) << 16);
    o.z = (uint32_t)f32_to_bf16(b.x) | ((uint32_t)f32_to_bf16(b.y) << 16);
    o.w = (uint32_t)f32_to_bf16(b.z) | ((uint32_t)f32_to_bf16(b.w) << 16);
    *reinterpret_cast<uint4*>(d) = o;
  }
};

template <>
struct Chunk<bf16_t, bf16_t, 8> {
  uint4 v;
  __device__ void load(const bf16_t* s) { v = *reinterpret_cast<const uint4*>(s); }
  __device__ void store(bf16_t* d) const { *reinterpret_cast<uint4*>(d) = v; }
};

template <>
struct Chunk<float, float, 1> {
  float v;
  __device__ void load(const float* s) { v = *s; }
  __device__ void store(float* d) const { *d = v; }
};

template <>
struct Chunk<float, bf16_t, 1> {
  float v;
  __device__ void load(const float* s) { v = *s; }
  __device__ void store(bf16_t* d) const { *d = f32_to_bf16(v); }
};

template <>
struct Chunk<bf16_t, bf16_t, 1> {
  bf16_t v;
  __device__ void load(const bf16_t* s) { v = *s; }
  __device__ void store(bf16_t* d) const { *d = v; }
};

// packed[l*kz + k] = conv(src[(gmap[l]-lo)*ld + k0 + k]), VO elements per chunk.
template <typename Tin, typename Tout, int VO>
__global__ __launch_bounds__(256) void k_gather(int64_t n, const int64_t* __restrict__ gmap,
                                                int64_t lo, const Tin* __restrict__ src,
                                                int64_t ld, int k0, int kz,
                                                Tout* __restrict__ dst) {
  const int chunks = kz / VO;
  const int64_t total = n * chunks;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x * kUnroll + threadIdx.x; base < total;
       base += stride) {
    Chunk<Tin, Tout, VO> c[kUnroll];
    int64_t at[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x;
      at[u] = i;
      if (i < total) {
        const int64_t l = i / chunks;
        const int ci = (int)(i - l * chunks);
        c[u].load(src + (gmap[l] - lo) * ld + k0 + (int64_t)ci * VO);
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (at[u] < total) {
        const int64_t l = at[u] / chunks;
        const int ci = (int)(at[u] - l * chunks);
        c[u].store(dst + l * kz + (int64_t)ci * VO);
      }
    }
  }
}

// dst[(gmap[l]-lo)*ld + k0 + k] += packed[l*kz + k]; VO elements per chunk.
template <int VO>
__global__ __launch_bounds__(256) void k_scatter_add(int64_t n, const int64_t* __restrict__ gmap,
                                                     int64_t lo, const float* __restrict__ packed,
                                                     int kz, float* __restrict__ dst, int64_t ld,
                                                     int k0) {
  using V = typename std::conditional<VO == 4, float4, float>::type;
  const int chunks = kz / VO;
  const int64_t total = n * chunks;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kUnroll;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x * kUnroll + threadIdx.x; base < total;
       base += stride) {
    V a[kUnroll], b[kUnroll];
    float* d[kUnroll];
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      const int64_t i = base + (int64_t)u * blockDim.x;
      d[u] = nullptr;
      if (i < total) {
        const int64_t l = i / chunks;
        const int ci = (int)(i - l * chunks);
        d[u] = dst + (gmap[l] - lo) * ld + k0 + (int64_t)ci * VO;
        a[u] = *reinterpret_cast<const V*>(d[u]);
        b[u] = *reinterpret_cast<const V*>(packed + l * kz + (int64_t)ci * VO);
      }
    }
#pragma unroll
    for (int u = 0; u < kUnroll; ++u) {
      if (d[u]) {
        V r = a[u];
        if constexpr (VO == 4) {
          r.x = a[u].x + b[u].x; r.y = a[u].y + b[u].y; r.z = a[u].z + b[u].z; r.w = a[u].w + b[u].w;
        } else {
          r = a[u] + b[u];
        }
        *reinterpret_cast<V*>(d[u]) = r;
      }
    }
  }
}

static unsigned grid_chunks(int64_t total) {
  int64_t b = (total + 256 * kUnroll - 1) / (256 * kUnroll);
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
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
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
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
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
