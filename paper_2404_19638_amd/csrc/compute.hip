// SDDMM / SpMM entry points: argument checks, variant choice and launch.
// The kernels and their design notes are in kernels.h; their instantiations
// are spread over inst_*.hip so they compile in parallel.
#include <mutex>

#include "kernels.h"

namespace spc3d {

#define SPC3D_EXTERN_LAUNCHERS(T, V)                                                          \
  extern template void launch_sddmm<T, V>(SPC3D_SDDMM_LAUNCH_ARGS);                            \
  extern template void launch_spmm<T, V, false>(SPC3D_SPMM_LAUNCH_ARGS);                      \
  extern template void launch_spmm<T, V, true>(SPC3D_SPMM_LAUNCH_ARGS);
SPC3D_EXTERN_LAUNCHERS(float, 4)
SPC3D_EXTERN_LAUNCHERS(float, 1)
SPC3D_EXTERN_LAUNCHERS(bf16_t, 8)
SPC3D_EXTERN_LAUNCHERS(bf16_t, 1)
#undef SPC3D_EXTERN_LAUNCHERS

namespace {

// Shared body of spc3d_spmm, spc3d_sddmm_spmm, spc3d_sddmm_spmm_static and
// spc3d_sddmm_spmm_scatter.  Y: where finished rows go; acc: kAccY / kAccOut
// bits; static_buf: d_buf is the library's own scratch array.
spc3d_status run_spmm(Plan* p, int transpose, const float* d_vals, const void* d_X,
                      spc3d_dtype x_t, int32_t kz, const YOut& Y, int acc, int variant,
                      void* d_buf, size_t buf_bytes, hipStream_t stream, const void* d_A,
                      float* d_out, bool static_buf = false) {
  const bool fused = d_A != nullptr;
  Shape sh;
  const bool al = aligned16(d_X) && aligned16(Y.base) && Y.ld % 4 == 0 &&
                  (!fused || aligned16(d_A));
  spc3d_status st = pick_shape(kz, x_t, al, variant, fused ? 2 : 1, p->nnz, &sh);
  if (st != SPC3D_OK) return st;
  const int64_t nitems = (p->nnz + sh.items - 1) / sh.items;
  const size_t need = (size_t)nitems * 2 * (size_t)kz * 4;
  if (buf_bytes < need) {
    if (static_buf)
      return fail(SPC3D_ERR_WORKSPACE,
                  "this call needs %zu bytes of scratch; the library's static scratch holds %zu "
                  "(use spc3d_sddmm_spmm with a caller buffer)", need, buf_bytes);
    return fail(SPC3D_ERR_WORKSPACE, "SpMM buffer %zu bytes < %zu required", buf_bytes, need);
  }
  const size_t lds = sh.window ? 0 : 4 * spmm_wave_lds(sh.items, sh.lanes, sh.nch, sh.vec, fused);
  if (lds > 65536) return fail(SPC3D_ERR_UNSUPPORTED, "variant needs %zu bytes of LDS", lds);
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
  const int64_t nblocks = (nitems + 3) / 4;
  Orient o = transpose ? p->csc() : p->csr();
  if (transpose == 2) o.vidx = nullptr;   // values already in column-major slot order
  float* carry = static_cast<float*>(d_buf);
#define SPC3D_RUN(T, V)                                                                        \
  do {                                                                                         \
    if (fused)                                                                                 \
      launch_spmm<T, V, true>(sh, stream, p->nnz, nitems, nblocks, o, d_vals, d_X, kz, Y, acc, \
                              carry, lds, d_A, d_out);                                         \
    else                                                                                       \
      launch_spmm<T, V, false>(sh, stream, p->nnz, nitems, nblocks, o, d_vals, d_X, kz, Y, acc,\
                               carry, lds, nullptr, nullptr);                                  \
  } while (0)
  if (x_t == SPC3D_F32) {
    if (sh.vec == 4) SPC3D_RUN(float, 4);
    else SPC3D_RUN(float, 1);
  } else {
    if (sh.vec == 8) SPC3D_RUN(bf16_t, 8);
    else SPC3D_RUN(bf16_t, 1);
  }
#undef SPC3D_RUN
  SPC3D_LAUNCHED(fused ? "sddmm_spmm" : "spmm");
  return SPC3D_OK;
}

// The kernels' accumulate bits for an output mode that applies to both outputs.
int acc_bits(int mode) { return mode == SPC3D_ACCUMULATE ? (kAccY | kAccOut) : 0; }

// Arguments common to the fused entry points.
spc3d_status check_fused_args(spc3d_plan h, Plan** p, spc3d_dtype ab_t, int32_t kz, int mode) {
  spc3d_status st = get_plan(h, p);
  if (st != SPC3D_OK) return st;
  if (ab_t != SPC3D_F32 && ab_t != SPC3D_BF16) return fail(SPC3D_ERR_INVALID_ARG, "bad ab_t");
  if (mode != SPC3D_OVERWRITE && mode != SPC3D_ACCUMULATE)
    return fail(SPC3D_ERR_INVALID_ARG, "bad mode");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "kz=%d outside [1,%d]", kz, kMaxKz);
  return SPC3D_OK;
}

// The scratch of spc3d_sddmm_spmm_static: the SpMM carries of one call, in a
// device array the library owns.  Each GPU the library runs on holds its own
// copy (kept until the process ends); host code reaches it only through the
// device address hipGetSymbolAddress gives with that GPU current.
static __device__ __align__(256) char scratch[SPC3D_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
spc3d_status static_scratch(void** out) {
  int dev = -1;
  SPC3D_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(SPC3D_ERR_UNSUPPORTED, "device %d beyond the %d the static scratch serves", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_addr[dev]) {
    void* addr = nullptr;
    SPC3D_HIP(hipGetSymbolAddress(&addr, HIP_SYMBOL(scratch)));
    if (!addr) return fail(SPC3D_ERR_HIP, "hipGetSymbolAddress gave no address for the scratch");
    g_scratch_addr[dev] = addr;
  }
  *out = g_scratch_addr[dev];
  return SPC3D_OK;
}

}  // namespace
}  // namespace spc3d

using namespace spc3d;

extern "C" {

spc3d_status spc3d_sddmm(spc3d_plan h, const float* d_vals, const void* d_A, const void* d_B,
                         spc3d_dtype ab_t, int32_t kz, float* d_out, int mode, int variant,
                         hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (ab_t != SPC3D_F32 && ab_t != SPC3D_BF16) return fail(SPC3D_ERR_INVALID_ARG, "bad ab_t");
  if (mode != SPC3D_OVERWRITE && mode != SPC3D_ACCUMULATE)
    return fail(SPC3D_ERR_INVALID_ARG, "bad mode");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "kz=%d outside [1,%d]", kz, kMaxKz);
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_A || !d_B || !d_out) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  Shape sh;
  st = pick_shape(kz, ab_t, aligned16(d_A) && aligned16(d_B), variant, 0, p->nnz, &sh);
  if (st != SPC3D_OK) return st;
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
  const int64_t nitems = (p->nnz + sh.items - 1) / sh.items;
  const int64_t nblocks = (nitems + 3) / 4;
  const Orient o = p->csr();
  const int acc = mode == SPC3D_ACCUMULATE;
  if (ab_t == SPC3D_F32) {
    if (sh.vec == 4)
      launch_sddmm<float, 4>(sh, stream, p->nnz, nitems, nblocks, o, d_vals, d_A, d_B, kz, d_out,
                             acc);
    else
      launch_sddmm<float, 1>(sh, stream, p->nnz, nitems, nblocks, o, d_vals, d_A, d_B, kz, d_out,
                             acc);
  } else {
    if (sh.vec == 8)
      launch_sddmm<bf16_t, 8>(sh, stream, p->nnz, nitems, nblocks, o, d_vals, d_A, d_B, kz,
                              d_out, acc);
    else
      launch_sddmm<bf16_t, 1>(sh, stream, p->nnz, nitems, nblocks, o, d_vals, d_A, d_B, kz,
                              d_out, acc);
  }
  SPC3D_LAUNCHED("sddmm");
  return SPC3D_OK;
}

spc3d_status spc3d_spmm_buffer_size(spc3d_plan h, int transpose, int32_t kz, int variant,
                                    size_t* bytes) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (!bytes) return fail(SPC3D_ERR_INVALID_ARG, "bytes is NULL");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "kz=%d outside [1,%d]", kz, kMaxKz);
  // The work-item size, and so the number of carries, depends on the shape a
  // call takes: the operand type, whether the operands are 16-byte aligned
  // and whether the pass is fused.  The size covers every shape that can run.
  int64_t items = 0;
  bool any = false;
  spc3d_status first = SPC3D_OK;
  for (int op = 1; op <= 2; ++op)
    for (int t = 0; t < 2; ++t)
      for (int al = 1; al >= 0; --al) {
        Shape sh;
        st = pick_shape(kz, t ? SPC3D_BF16 : SPC3D_F32, al != 0, variant, op, p->nnz, &sh);
        if (st == SPC3D_OK) {
          any = true;
          const int64_t n = (p->nnz + sh.items - 1) / sh.items;
          items = n > items ? n : items;
        } else if (first == SPC3D_OK) {
          first = st;
        }
      }
  if (!any) return first;
  *bytes = (size_t)(items > 0 ? items : 1) * 2 * (size_t)kz * 4;
  return SPC3D_OK;
}

spc3d_status spc3d_spmm(spc3d_plan h, int transpose, const float* d_vals, const void* d_X,
                        spc3d_dtype x_t, int32_t kz, float* d_Y, int mode, int variant,
                        void* d_buf, size_t buf_bytes, hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (transpose < 0 || transpose > 2) return fail(SPC3D_ERR_INVALID_ARG, "bad transpose");
  if (transpose && !(p->flags & SPC3D_BUILD_CSC))
    return fail(SPC3D_ERR_INVALID_ARG, "transposed SpMM needs a plan built with BUILD_CSC");
  if (x_t != SPC3D_F32 && x_t != SPC3D_BF16) return fail(SPC3D_ERR_INVALID_ARG, "bad x_t");
  if (mode != SPC3D_OVERWRITE && mode != SPC3D_ACCUMULATE)
    return fail(SPC3D_ERR_INVALID_ARG, "bad mode");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "kz=%d outside [1,%d]", kz, kMaxKz);
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_X || !d_Y || !d_buf) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_buf) & 255u)
    return fail(SPC3D_ERR_INVALID_ARG, "buffer must be 256-byte aligned");
  const YOut Y{d_Y, nullptr, 0, kz, 0};
  return run_spmm(p, transpose, d_vals, d_X, x_t, kz, Y, acc_bits(mode), variant, d_buf,
                  buf_bytes, stream, nullptr, nullptr);
}

spc3d_status spc3d_sddmm_spmm(spc3d_plan h, const float* d_vals, const void* d_A, const void* d_B,
                              spc3d_dtype ab_t, int32_t kz, float* d_out, float* d_Y, int mode,
                              int variant, void* d_buf, size_t buf_bytes, hipStream_t stream) {
  Plan* p;
  spc3d_status st = check_fused_args(h, &p, ab_t, kz, mode);
  if (st != SPC3D_OK) return st;
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_A || !d_B || !d_out || !d_Y || !d_buf) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_buf) & 255u)
    return fail(SPC3D_ERR_INVALID_ARG, "buffer must be 256-byte aligned");
  const YOut Y{d_Y, nullptr, 0, kz, 0};
  return run_spmm(p, 0, d_vals, d_B, ab_t, kz, Y, acc_bits(mode), variant, d_buf, buf_bytes,
                  stream, d_A, d_out);
}

spc3d_status spc3d_sddmm_spmm_static(spc3d_plan h, const float* d_vals, const void* d_A,
                                     const void* d_B, spc3d_dtype ab_t, int32_t kz, float* d_out,
                                     float* d_Y, int mode, int variant, hipStream_t stream) {
  Plan* p;
  spc3d_status st = check_fused_args(h, &p, ab_t, kz, mode);
  if (st != SPC3D_OK) return st;
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_A || !d_B || !d_out || !d_Y) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  void* buf = nullptr;
  st = static_scratch(&buf);
  if (st != SPC3D_OK) return st;
  const YOut Y{d_Y, nullptr, 0, kz, 0};
  return run_spmm(p, 0, d_vals, d_B, ab_t, kz, Y, acc_bits(mode), variant, buf,
                  SPC3D_STATIC_SCRATCH_BYTES, stream, d_A, d_out, true);
}

spc3d_status spc3d_sddmm_spmm_scatter(spc3d_plan h, const float* d_vals, const void* d_A,
                                      const void* d_B, spc3d_dtype ab_t, int32_t kz, float* d_out,
                                      int out_mode, float* d_dst, int64_t ld_dst, int32_t k0,
                                      int variant, void* d_buf, size_t buf_bytes,
                                      hipStream_t stream) {
  Plan* p;
  spc3d_status st = check_fused_args(h, &p, ab_t, kz, out_mode);
  if (st != SPC3D_OK) return st;
  if (k0 < 0 || ld_dst < (int64_t)k0 + kz)
    return fail(SPC3D_ERR_INVALID_ARG, "k0=%d kz=%d do not fit ld_dst=%lld", k0, kz,
                (long long)ld_dst);
  if (p->nnz == 0) return SPC3D_OK;
  if (!d_A || !d_B || !d_out || !d_dst || !d_buf) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_buf) & 255u)
    return fail(SPC3D_ERR_INVALID_ARG, "buffer must be 256-byte aligned");
  const YOut Y{d_dst + k0, p->gmap_r, p->row_lo, ld_dst, p->R};
  const int acc = kAccY | (out_mode == SPC3D_ACCUMULATE ? kAccOut : 0);
  return run_spmm(p, 0, d_vals, d_B, ab_t, kz, Y, acc, variant, d_buf, buf_bytes, stream, d_A,
                  d_out);
}

spc3d_status spc3d_variant_check(int op, int32_t kz, spc3d_dtype ab_t, int variant) {
  if (op < SPC3D_OP_SDDMM || op > SPC3D_OP_SDDMM_SPMM) return fail(SPC3D_ERR_INVALID_ARG, "bad op %d", op);
  if (ab_t != SPC3D_F32 && ab_t != SPC3D_BF16) return fail(SPC3D_ERR_INVALID_ARG, "bad ab_t");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "kz=%d outside [1,%d]", kz, kMaxKz);
  Shape sh;
  return pick_shape(kz, ab_t, true, variant, op, 0, &sh);
}

}  // extern "C"
