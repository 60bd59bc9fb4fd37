// The spectral loss of Eq. 8 and its gradient, for inverse rendering against
// targets that cannot be aligned pixel by pixel.  With F the unnormalised 2-D
// DFT and eps > 0 inside the logarithms,
//   A(k) = log(|F(I)(k)| + eps) - log(|F(T)(k)| + eps),   L = (1/HW) sum_k A(k)^2,
//   dL/dI = Re(DFT(g)),   g(k) = (2/HW) A(k) conj(F(k)) / (|F(k)| (|F(k)| + eps))
// (g = 0 on an empty bin).  Three LDS-staged Stockham passes on the blocked band
// layout with every column in band:
//   k_spec_rows      image rows -> row DFTs                                  -> band
//   k_spec_cols      column DFTs, A, per-column sums of A^2, g, column DFT of g -> band
//                    (or, for the target, log(|F| + eps) stored column-major)
//   k_spec_grad      row DFTs of the band, real part                         -> dL/dI
//   k_spec_sum       L = fixed-order sum of the column sums / HW
#include <hip/hip_runtime.h>

#include "fft_common.h"
#include "osog_internal.h"

namespace osog {

__device__ __forceinline__ size_t spec_at(int i, int b, int W, int rb) {
  return ((size_t)(i / rb) * W + b) * rb + (i % rb);
}

template <int LOGW>
__global__ void __launch_bounds__(kThreads) k_spec_rows(const float* __restrict__ img, float2* __restrict__ band,
                                                        const float2* __restrict__ tw) {
  constexpr int W = 1 << LOGW, RPB = rows_per_fft_block(W), RB = rows_per_block(W);
  __shared__ __align__(16) float2 buf[fft_lds_f2(RPB * W)];
  const int t = threadIdx.x, row0 = blockIdx.x * RPB;
  gather_lds<8>(
      RPB * W, [&](int idx) { return make_float2(img[(size_t)row0 * W + idx], 0.0f); },
      [&](int idx, float2 v) { buf[idx] = v; });
  __syncthreads();
  Stages<W, RPB, -1, 1, LOGW>::run(buf, tw);
  for (int idx = t; idx < RPB * W; idx += kThreads) {
    const int b = idx / RPB, r = idx - b * RPB;
    band[spec_at(row0 + r, b, W, RB)] = buf[r * W + b];
  }
}

// target_out != null: store log(|F| + eps) column-major (k = b * H + ky) and stop.
// Otherwise compare with target (same layout), write the column's sum of A^2 and,
// when with_grad, replace the column by the column DFT of g.
template <int LOGH>
__global__ void __launch_bounds__(kThreads) k_spec_cols(float2* __restrict__ band, int W,
                                                        const float* __restrict__ target,
                                                        float* __restrict__ target_out, float eps, int with_grad,
                                                        double* __restrict__ colsum, const float2* __restrict__ tw) {
#pragma clang fp contract(off)
  constexpr int H = 1 << LOGH;
  __shared__ float2 buf[fft_lds_f2(H)];
  __shared__ double red[kThreads];
  const int t = threadIdx.x, b = blockIdx.x, RB = W >= 1024 ? 8192 / W : 8;
  gather_lds<8>(
      H, [&](int i) { return band[spec_at(i, b, W, RB)]; }, [&](int i, float2 v) { buf[i] = v; });
  __syncthreads();
  Stages<H, 1, -1, 1, LOGH>::run(buf, tw);
  if (target_out) {
    for (int m = t; m < H; m += kThreads) {
      const float2 f = buf[m];
      target_out[(size_t)b * H + m] = logf(sqrtf(f.x * f.x + f.y * f.y) + eps);
    }
    return;
  }
  const float g_scale = 2.0f / ((float)H * (float)W);
  double part = 0.0;
  for (int m = t; m < H; m += kThreads) {
    const float2 f = buf[m];
    const float mag = sqrtf(f.x * f.x + f.y * f.y);
    const float A = logf(mag + eps) - target[(size_t)b * H + m];
    part += (double)A * (double)A;
    if (with_grad) {
      const float s = mag > 0.0f ? g_scale * A / (mag * (mag + eps)) : 0.0f;
      buf[m] = make_float2(s * f.x, -s * f.y);  // s conj(F)
    }
  }
  const double cs = block_sum(part, red);  // its barriers also order buf for the stages
  if (t == 0) colsum[b] = cs;
  if (!with_grad) return;
  Stages<H, 1, -1, 1, LOGH>::run(buf, tw);
  for (int i = t; i < H; i += kThreads) band[spec_at(i, b, W, RB)] = buf[i];
}

template <int LOGW>
__global__ void __launch_bounds__(kThreads) k_spec_grad(const float2* __restrict__ band, float* __restrict__ grad,
                                                        const float2* __restrict__ tw) {
  constexpr int W = 1 << LOGW, RPB = rows_per_fft_block(W), RB = rows_per_block(W);
  __shared__ __align__(16) float2 buf[fft_lds_f2(RPB * W)];
  const int t = threadIdx.x, row0 = blockIdx.x * RPB;
  gather_lds<8>(
      RPB * W,
      [&](int idx) {
        const int b = idx / RPB, r = idx - b * RPB;
        return band[spec_at(row0 + r, b, W, RB)];
      },
      [&](int idx, float2 v) {
        const int b = idx / RPB, r = idx - b * RPB;
        buf[r * W + b] = v;
      });
  __syncthreads();
  Stages<W, RPB, -1, 1, LOGW>::run(buf, tw);
  for (int idx = t; idx < RPB * W; idx += kThreads) grad[(size_t)row0 * W + idx] = buf[idx].x;
}

__global__ void __launch_bounds__(kThreads) k_spec_sum(const double* __restrict__ colsum, int W, double inv_n,
                                                       float* __restrict__ loss) {
  __shared__ double red[kThreads];
  const int t = threadIdx.x;
  double s = 0.0;
  for (int b = t; b < W; b += kThreads) s += colsum[b];
  red[t] = s;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (t < st) red[t] += red[t + st];
    __syncthreads();
  }
  if (t == 0) loss[0] = (float)(red[0] * inv_n);
}

#define OSOG_SIZE_SWITCH(LOG, CALL) \
  switch (LOG) {                    \
    case 5: CALL(5); break;         \
    case 6: CALL(6); break;         \
    case 7: CALL(7); break;         \
    case 8: CALL(8); break;         \
    case 9: CALL(9); break;         \
    case 10: CALL(10); break;       \
    case 11: CALL(11); break;       \
    case 12: CALL(12); break;       \
    default: return hipErrorInvalidValue; \
  }

static int ilog2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

size_t spectral_workspace_bytes(int H, int W) {
  return (((size_t)H * W * sizeof(float2) + 255) / 256) * 256 + (size_t)W * sizeof(double);
}

// target_out != null: the target's log amplitudes.  Otherwise the loss into
// loss (device float[1]) and, if grad != null, dL/dimage.
hipError_t spectral_run(int H, int W, const float* img, const float* target, float* target_out, float eps,
                        float* loss, float* grad, void* ws, const float2* tw, hipStream_t s) {
  float2* band = static_cast<float2*>(ws);
  double* colsum = reinterpret_cast<double*>(static_cast<char*>(ws) +
                                             (((size_t)H * W * sizeof(float2) + 255) / 256) * 256);
  const int lh = ilog2i(H), lw = ilog2i(W);
  const int groups = H / rows_per_fft_block(W);
  const int with_grad = grad != nullptr;
#define K(LG) hipLaunchKernelGGL(k_spec_rows<LG>, dim3(groups), dim3(kThreads), 0, s, img, band, tw)
  OSOG_SIZE_SWITCH(lw, K)
#undef K
#define K(LG) hipLaunchKernelGGL(k_spec_cols<LG>, dim3(W), dim3(kThreads), 0, s, band, W, target, target_out, eps, \
                                 with_grad, colsum, tw)
  OSOG_SIZE_SWITCH(lh, K)
#undef K
  if (target_out) return hipGetLastError();
  hipLaunchKernelGGL(k_spec_sum, dim3(1), dim3(kThreads), 0, s, colsum, W, 1.0 / ((double)H * (double)W), loss);
  if (with_grad) {
#define K(LG) hipLaunchKernelGGL(k_spec_grad<LG>, dim3(groups), dim3(kThreads), 0, s, band, grad, tw)
    OSOG_SIZE_SWITCH(lw, K)
#undef K
  }
  return hipGetLastError();
}

}  // namespace osog
