// Learned kernel-variant selector (an extension; the paper has no such part):
// per-block sparsity features and the small multilayer perceptron that maps
// them to predicted relative run times of the SDDMM / SpMM kernel variants.
//
// MLP layers are dense, Y = act(X W^T + b), with X [n x fin] and W [fout x fin]
// row-major.  Sizes are tiny (fin, fout <= 1024, in practice <= 64), so one
// thread computes one output element.  The weight gradients, reductions over
// the batch, are summed in blocks of 32 rows and then over the blocks in a
// fixed order, so every kernel here is deterministic.
#include <cmath>

#include "internal.h"

namespace spc3d {

constexpr int kBins = 16;  // row-length classes [2^b, 2^(b+1)), the last open-ended

__global__ __launch_bounds__(256) void k_row_hist(int64_t nrows, const int32_t* __restrict__ ptr,
                                                  unsigned long long* __restrict__ hist,
                                                  int* __restrict__ maxlen) {
  __shared__ unsigned long long h[kBins];
  __shared__ int mx;
  if (threadIdx.x < kBins) h[threadIdx.x] = 0;
  if (threadIdx.x == 0) mx = 0;
  __syncthreads();
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    const int len = ptr[r + 1] - ptr[r];
    if (len > 0) {
      int b = 31 - __clz(len);
      b = b < kBins ? b : kBins - 1;
      atomicAdd(&h[b], (unsigned long long)len);
      atomicMax(&mx, len);
    }
  }
  __syncthreads();
  if (threadIdx.x < kBins && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
  if (threadIdx.x == 0 && mx) atomicMax(maxlen, mx);
}

__device__ inline float lg(double x) { return (float)log2(x > 1.0 ? x : 1.0); }

// Feature vector (SPC3D_NFEAT entries), every entry O(1):
//   [0, 16)  fraction of the entries lying in rows of length [2^b, 2^(b+1))
//   16 log2(longest row) / 16      17 log2(rows) / 16     18 log2(columns) / 16
//   19 log2(nnz) / 24              20 log2(nnz / rows) / 8
//   21 log2(kz) / 8                22 1 for BF16 operands, else 0
__global__ void k_feat_finish(const unsigned long long* __restrict__ hist,
                              const int* __restrict__ maxlen, int64_t nnz, int64_t nrows,
                              int64_t ncols, int kz, int bf16, float* __restrict__ out) {
  const int i = threadIdx.x;
  if (i < kBins) out[i] = nnz > 0 ? (float)((double)hist[i] / (double)nnz) : 0.f;
  if (i == 16) out[i] = lg((double)maxlen[0]) / 16.f;
  if (i == 17) out[i] = lg((double)nrows) / 16.f;
  if (i == 18) out[i] = lg((double)ncols) / 16.f;
  if (i == 19) out[i] = lg((double)nnz) / 24.f;
  if (i == 20) out[i] = nrows > 0 ? lg((double)nnz / (double)nrows) / 8.f : 0.f;
  if (i == 21) out[i] = lg((double)kz) / 8.f;
  if (i == 22) out[i] = bf16 ? 1.f : 0.f;
}

__global__ void k_clear_words(unsigned long long* p, int n) {
  if ((int)threadIdx.x < n) p[threadIdx.x] = 0;
}

// Y = act(X W^T + b); relu != 0 applies max(0, .).  b may be NULL.
__global__ __launch_bounds__(256) void k_linear_fwd(int n, int fin, int fout,
                                                    const float* __restrict__ X,
                                                    const float* __restrict__ W,
                                                    const float* __restrict__ b,
                                                    float* __restrict__ Y, int relu) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * fout) return;
  const int r = (int)(i / fout), o = (int)(i % fout);
  const float* x = X + (int64_t)r * fin;
  const float* w = W + (int64_t)o * fin;
  float acc = 0.f;
  for (int k = 0; k < fin; ++k) acc = fmaf(x[k], w[k], acc);
  if (b) acc += b[o];
  Y[i] = (relu && !(acc > 0.f)) ? 0.f : acc;
}

// G = dY where Y > 0, else 0 (the ReLU's derivative taken as 0 at 0).
__global__ void k_relu_mask(int64_t n, const float* __restrict__ Y, const float* __restrict__ dY,
                            float* __restrict__ G) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    G[i] = Y[i] > 0.f ? dY[i] : 0.f;
}

// dX = G W   ([n x fout] times [fout x fin]).
__global__ __launch_bounds__(256) void k_linear_dx(int n, int fin, int fout,
                                                   const float* __restrict__ G,
                                                   const float* __restrict__ W,
                                                   float* __restrict__ dX) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)n * fin) return;
  const int r = (int)(i / fin), k = (int)(i % fin);
  const float* g = G + (int64_t)r * fout;
  float acc = 0.f;
  for (int o = 0; o < fout; ++o) acc = fmaf(g[o], W[(int64_t)o * fin + k], acc);
  dX[i] = acc;
}

// Partial weight gradients of the 32-row block blockIdx.y:
//   P[blk][o][k] = sum_r G[r][o] X[r][k],   Pb[blk][o] = sum_r G[r][o].
__global__ __launch_bounds__(256) void k_linear_dw_part(int n, int fin, int fout,
                                                        const float* __restrict__ G,
                                                        const float* __restrict__ X,
                                                        float* __restrict__ P,
                                                        float* __restrict__ Pb) {
  const int blk = blockIdx.y;
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= (int64_t)fout * (fin + 1)) return;
  const int o = (int)(i / (fin + 1)), k = (int)(i % (fin + 1));
  const int r0 = blk * 32, r1 = (r0 + 32 < n) ? r0 + 32 : n;
  float acc = 0.f;
  if (k < fin) {
    for (int r = r0; r < r1; ++r) acc = fmaf(G[(int64_t)r * fout + o], X[(int64_t)r * fin + k], acc);
    P[((int64_t)blk * fout + o) * fin + k] = acc;
  } else {
    for (int r = r0; r < r1; ++r) acc += G[(int64_t)r * fout + o];
    Pb[(int64_t)blk * fout + o] = acc;
  }
}

__global__ __launch_bounds__(256) void k_linear_dw_sum(int nblk, int fin, int fout,
                                                       const float* __restrict__ P,
                                                       const float* __restrict__ Pb,
                                                       float* __restrict__ dW,
                                                       float* __restrict__ db) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t nw = (int64_t)fout * fin;
  if (i < nw) {
    float acc = 0.f;
    for (int b = 0; b < nblk; ++b) acc += P[(int64_t)b * nw + i];
    dW[i] = acc;
  } else if (i < nw + fout && db) {
    const int o = (int)(i - nw);
    float acc = 0.f;
    for (int b = 0; b < nblk; ++b) acc += Pb[(int64_t)b * fout + o];
    db[o] = acc;
  }
}

// Masked mean squared error over n entries, one block, sums in a fixed order:
//   loss = sum m (p - t)^2 / sum m,    dP = 2 m (p - t) / sum m.
__global__ __launch_bounds__(256) void k_mse(int64_t n, const float* __restrict__ P,
                                             const float* __restrict__ T,
                                             const float* __restrict__ M, float* __restrict__ dP,
                                             float* __restrict__ loss) {
  __shared__ float s_l[256], s_c[256];
  float l = 0.f, c = 0.f;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const float d = P[i] - T[i];
    l = fmaf(M[i] * d, d, l);
    c += M[i];
  }
  s_l[threadIdx.x] = l;
  s_c[threadIdx.x] = c;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      s_l[threadIdx.x] += s_l[threadIdx.x + s];
      s_c[threadIdx.x] += s_c[threadIdx.x + s];
    }
    __syncthreads();
  }
  const float cnt = s_c[0] > 0.f ? s_c[0] : 1.f;
  if (threadIdx.x == 0 && loss) loss[0] = s_l[0] / cnt;
  const float sc = 2.f / cnt;
  for (int64_t i = threadIdx.x; i < n; i += 256) dP[i] = sc * M[i] * (P[i] - T[i]);
}

// One Adam step (Kingma and Ba, 2015, Algorithm 1); c1, c2 are the bias
// corrections 1 - beta1^t and 1 - beta2^t of step t.
__global__ void k_adam(int64_t n, float* __restrict__ w, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// idx[r] = the column o < m with mask[r][o] != 0 and the least P[r][o] (the
// first such column on ties); -1 when the row's mask is all zero.  With pref
// in [0, m): pref instead, when it is allowed and P[r][pref] <= least + margin
// (FP32 sum).
__global__ void k_masked_argmin(int n, int m, const float* __restrict__ P,
                                const float* __restrict__ M, int pref, float margin,
                                int32_t* __restrict__ idx) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  int best = -1;
  float bv = 0.f;
  for (int o = 0; o < m; ++o) {
    if (M[(int64_t)r * m + o] == 0.f) continue;
    const float v = P[(int64_t)r * m + o];
    if (best < 0 || v < bv) {
      best = o;
      bv = v;
    }
  }
  if (best >= 0 && pref >= 0 && M[(int64_t)r * m + pref] != 0.f &&
      P[(int64_t)r * m + pref] <= bv + margin)
    best = pref;
  idx[r] = best;
}

namespace {
// Grids here are not grid-stride: these limits keep every launch within
// 65535 blocks per dimension.
constexpr int kMaxWidth = 1024;
constexpr int kMaxRows = 1 << 20;
unsigned blocks_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b < 1) b = 1;
  if (b > 65535) b = 65535;
  return (unsigned)b;
}
spc3d_status check_dims(int n, int fin, int fout) {
  if (n < 0 || n > kMaxRows || fin < 1 || fout < 1 || fin > kMaxWidth || fout > kMaxWidth ||
      (int64_t)n * (fin > fout ? fin : fout) > (int64_t)65535 * 256)
    return fail(SPC3D_ERR_INVALID_ARG, "bad layer sizes n=%d fin=%d fout=%d", n, fin, fout);
  return SPC3D_OK;
}
int64_t dw_blocks(int n) { return n > 0 ? (n + 31) / 32 : 1; }
}  // namespace

}  // namespace spc3d

using namespace spc3d;

extern "C" {

spc3d_status spc3d_plan_features(spc3d_plan h, int transpose, int32_t kz, spc3d_dtype ab_t,
                                 float* d_out, void* d_buf, size_t buf_bytes,
                                 hipStream_t stream) {
  Plan* p;
  spc3d_status st = get_plan(h, &p);
  if (st != SPC3D_OK) return st;
  if (transpose != 0 && transpose != 1) return fail(SPC3D_ERR_INVALID_ARG, "transpose must be 0 or 1");
  if (transpose && !(p->flags & SPC3D_BUILD_CSC))
    return fail(SPC3D_ERR_INVALID_ARG, "column features need a plan built with SPC3D_BUILD_CSC");
  if (kz < 1 || kz > kMaxKz) return fail(SPC3D_ERR_INVALID_ARG, "bad kz %d", kz);
  if (ab_t != SPC3D_F32 && ab_t != SPC3D_BF16) return fail(SPC3D_ERR_INVALID_ARG, "bad dtype");
  if (!d_out || !d_buf) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_buf) & 7u)
    return fail(SPC3D_ERR_INVALID_ARG, "buffer must be 8-byte aligned");
  if (buf_bytes < SPC3D_FEATURES_BUFFER_BYTES)
    return fail(SPC3D_ERR_WORKSPACE, "features buffer needs %d bytes", SPC3D_FEATURES_BUFFER_BYTES);
  DeviceGuard dg;
  st = dg.enter(p);
  if (st != SPC3D_OK) return st;
  SPC3D_DEBUG_CHECK(p, stream);
  unsigned long long* hist = static_cast<unsigned long long*>(d_buf);
  int* mx = reinterpret_cast<int*>(hist + kBins);
  const Orient o = transpose ? p->csc() : p->csr();
  hipLaunchKernelGGL(k_clear_words, dim3(1), dim3(64), 0, stream, hist, kBins + 1);
  if (o.nrows > 0) {
    unsigned nb = blocks_for(o.nrows);
    if (nb > 1024) nb = 1024;
    hipLaunchKernelGGL(k_row_hist, dim3(nb), dim3(256), 0, stream, o.nrows, o.ptr, hist, mx);
  }
  hipLaunchKernelGGL(k_feat_finish, dim3(1), dim3(64), 0, stream, hist, mx, o.nnz, o.nrows,
                     o.ncols, (int)kz, ab_t == SPC3D_BF16 ? 1 : 0, d_out);
  SPC3D_LAUNCHED("spc3d_plan_features");
  return SPC3D_OK;
}

spc3d_status spc3d_mlp_linear_fwd(int n, int fin, int fout, const float* d_X, const float* d_W,
                                  const float* d_b, float* d_Y, int relu, hipStream_t stream) {
  spc3d_status st = check_dims(n, fin, fout);
  if (st != SPC3D_OK) return st;
  if (n == 0) return SPC3D_OK;
  if (!d_X || !d_W || !d_Y) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  hipLaunchKernelGGL(k_linear_fwd, dim3(blocks_for((int64_t)n * fout)), dim3(256), 0, stream, n,
                     fin, fout, d_X, d_W, d_b, d_Y, relu);
  SPC3D_LAUNCHED("spc3d_mlp_linear_fwd");
  return SPC3D_OK;
}

spc3d_status spc3d_mlp_linear_bwd_buffer_size(int n, int fin, int fout, size_t* bytes) {
  spc3d_status st = check_dims(n, fin, fout);
  if (st != SPC3D_OK) return st;
  if (!bytes) return fail(SPC3D_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = (size_t)(dw_blocks(n) * fout * (int64_t)(fin + 1) + (int64_t)n * fout) * sizeof(float);
  return SPC3D_OK;
}

spc3d_status spc3d_mlp_linear_bwd(int n, int fin, int fout, const float* d_X, const float* d_W,
                                  const float* d_Y, const float* d_dY, int relu, float* d_dX,
                                  float* d_dW, float* d_db, void* d_buf, size_t buf_bytes,
                                  hipStream_t stream) {
  spc3d_status st = check_dims(n, fin, fout);
  if (st != SPC3D_OK) return st;
  if (!d_W || !d_dW || !d_buf || (n > 0 && (!d_X || !d_dY)) || (relu && n > 0 && !d_Y))
    return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  if (reinterpret_cast<uintptr_t>(d_buf) & 3u)
    return fail(SPC3D_ERR_INVALID_ARG, "buffer must be 4-byte aligned");
  size_t need = 0;
  spc3d_mlp_linear_bwd_buffer_size(n, fin, fout, &need);
  if (buf_bytes < need) return fail(SPC3D_ERR_WORKSPACE, "MLP backward buffer too small");
  const int64_t nblk = dw_blocks(n);
  float* P = static_cast<float*>(d_buf);
  float* Pb = P + nblk * fout * fin;
  float* G = Pb + nblk * fout;
  const float* g = d_dY;
  if (n > 0) {
    if (relu) {
      hipLaunchKernelGGL(k_relu_mask, dim3(blocks_for((int64_t)n * fout)), dim3(256), 0, stream,
                         (int64_t)n * fout, d_Y, d_dY, G);
      g = G;
    }
    if (d_dX)
      hipLaunchKernelGGL(k_linear_dx, dim3(blocks_for((int64_t)n * fin)), dim3(256), 0, stream, n,
                         fin, fout, g, d_W, d_dX);
    hipLaunchKernelGGL(k_linear_dw_part, dim3(blocks_for((int64_t)fout * (fin + 1)), (unsigned)nblk),
                       dim3(256), 0, stream, n, fin, fout, g, d_X, P, Pb);
  }
  hipLaunchKernelGGL(k_linear_dw_sum, dim3(blocks_for((int64_t)fout * fin + fout)), dim3(256), 0,
                     stream, n > 0 ? (int)nblk : 0, fin, fout, P, Pb, d_dW, d_db);
  SPC3D_LAUNCHED("spc3d_mlp_linear_bwd");
  return SPC3D_OK;
}

spc3d_status spc3d_mlp_mse(int64_t n, const float* d_P, const float* d_T, const float* d_mask,
                           float* d_dP, float* d_loss, hipStream_t stream) {
  if (n < 0) return fail(SPC3D_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && (!d_P || !d_T || !d_mask || !d_dP)) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  hipLaunchKernelGGL(k_mse, dim3(1), dim3(256), 0, stream, n, d_P, d_T, d_mask, d_dP, d_loss);
  SPC3D_LAUNCHED("spc3d_mlp_mse");
  return SPC3D_OK;
}

spc3d_status spc3d_mlp_adam(int64_t n, float* d_w, const float* d_g, float* d_m, float* d_v,
                            float lr, float beta1, float beta2, float eps, int step,
                            hipStream_t stream) {
  if (n < 0 || step < 1 || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) ||
      !(eps > 0.f))
    return fail(SPC3D_ERR_INVALID_ARG, "bad Adam arguments");
  if (n == 0) return SPC3D_OK;
  if (!d_w || !d_g || !d_m || !d_v) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  // Bias corrections 1 - beta^t, formed on the host in double precision.
  const float c1 = (float)(1.0 - std::pow((double)beta1, (double)step));
  const float c2 = (float)(1.0 - std::pow((double)beta2, (double)step));
  hipLaunchKernelGGL(k_adam, dim3(blocks_for(n)), dim3(256), 0, stream, n, d_w, d_g, d_m, d_v, lr,
                     beta1, beta2, eps, c1, c2);
  SPC3D_LAUNCHED("spc3d_mlp_adam");
  return SPC3D_OK;
}

spc3d_status spc3d_mlp_masked_argmin(int n, int m, const float* d_P, const float* d_mask,
                                     int32_t pref, float margin, int32_t* d_idx,
                                     hipStream_t stream) {
  if (n < 0 || m < 1) return fail(SPC3D_ERR_INVALID_ARG, "bad sizes n=%d m=%d", n, m);
  if (pref < -1 || pref >= m) return fail(SPC3D_ERR_INVALID_ARG, "pref=%d outside [-1,%d)", pref, m);
  if (!(margin >= 0.f && margin <= 3.4e38f))
    return fail(SPC3D_ERR_INVALID_ARG, "margin must be finite and >= 0");
  if (n == 0) return SPC3D_OK;
  if (!d_P || !d_mask || !d_idx) return fail(SPC3D_ERR_INVALID_ARG, "NULL buffer");
  hipLaunchKernelGGL(k_masked_argmin, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, n,
                     m, d_P, d_mask, pref, margin, d_idx);
  SPC3D_LAUNCHED("spc3d_mlp_masked_argmin");
  return SPC3D_OK;
}

}  // extern "C"
