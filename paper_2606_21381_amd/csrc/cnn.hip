// Learned initializer: a small BF16 convolutional network on the MFMA matrix
// cores with FP32 accumulation, trained on frames the renderer itself
// produces, that regresses the global optical parameters (dn, defocus, DIC
// shear, bias) from a DIC image.
//
// Network (3x3 convolutions, padding 1, bias + ReLU, activations NHWC BF16):
//   1 -> 32 /2, 32 -> 32, 32 -> 64 /2, 64 -> 64, 64 -> 128 /2, 128 -> 128 /2,
//   global average pool, dense 128 -> 64 (ReLU), dense 64 -> 4.
// Every convolution -- forward, input gradient (dgrad) and weight gradient
// (wgrad) -- is an implicit GEMM whose operand tiles are gathered from the
// activations into LDS as BF16 and multiplied with v_mfma_f32_16x16x32_bf16:
//   forward  C[pix][co]  = sum_k  im2col(x)[pix][k]            W[k][co],  k = (ky,kx,ci)
//   dgrad    C[pix][ci]  = sum_k  col(gz)[pix][k]              W^T[k][ci], k = (ky,kx,co)
//   wgrad    C[k][co]    = sum_pix im2col(x)[pix][k]^T         gz[pix][co]  (split over pix)
// with gz = dL/d(output) masked by ReLU (output > 0).  In training the wgrad GEMM
// has one more row, of ones in im2col(x)^T, whose product row is the bias gradient
// sum_pix gz[pix][co].  The wgrad's split-K partial sums are reduced in a fixed
// order, so training is deterministic.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "osog_internal.h"

namespace osog {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t f2bf(float f) {  // round to nearest even
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)((u >> 16) | ((u & 0xFFFFu) ? 0x40u : 0u));
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct ConvGeom {
  int B, Hi, Wi, Ci, Ho, Wo, Co, stride;
};

enum ConvMode { CONV_FWD = 0, CONV_DGRAD = 1, CONV_WGRAD = 2 };

// Gathers for the three GEMM views.  Activations / gradients are NHWC BF16;
// weights are [ky][kx][ci][co] BF16.
struct ConvArgs {
  ConvGeom g;
  const uint16_t* x;      // layer input activations   [B][Hi][Wi][Ci]
  const uint16_t* y;      // layer output activations  [B][Ho][Wo][Co] (ReLU mask for dgrad/wgrad)
  const uint16_t* gy;     // dL/d(output)               [B][Ho][Wo][Co]
  const uint16_t* w;      // weights                    [3][3][Ci][Co]
  const float* bias;      // [Co] (forward)
  uint16_t* out_bf16;     // forward: activations; dgrad: dL/d(input) [B][Hi][Wi][Ci]
  float* out_f32;         // wgrad: partials [split][9 Ci][Co]
  int M, N, K;            // GEMM sizes
  int k_chunk;            // wgrad: pixels per split
};

__device__ __forceinline__ float relu_mask_grad(const ConvArgs& a, int64_t pix, int co) {
  const int64_t at = pix * a.g.Co + co;
  return a.y[at] != 0 && !(a.y[at] & 0x8000u) ? bf2f(a.gy[at]) : 0.0f;
}

// A operand element (row m, column k) of the GEMM.
template <int MODE>
__device__ __forceinline__ uint16_t gather_a(const ConvArgs& a, int m, int k) {
  const ConvGeom& g = a.g;
  if (MODE == CONV_FWD) {
    if (k >= 9 * g.Ci) return 0;
    const int hw = g.Ho * g.Wo, b = m / hw, r = m - b * hw, oy = r / g.Wo, ox = r - oy * g.Wo;
    const int tap = k / g.Ci, ci = k - tap * g.Ci, ky = tap / 3, kx = tap - ky * 3;
    const int iy = oy * g.stride - 1 + ky, ix = ox * g.stride - 1 + kx;
    if (iy < 0 || iy >= g.Hi || ix < 0 || ix >= g.Wi) return 0;
    return a.x[(((int64_t)b * g.Hi + iy) * g.Wi + ix) * g.Ci + ci];
  } else if (MODE == CONV_DGRAD) {
    // dL/dx[b,y,x,ci] = sum over (ky,kx,co) of gz[b,oy,ox,co] W[ky,kx,ci,co], y = oy*s - 1 + ky
    const int hw = g.Hi * g.Wi, b = m / hw, r = m - b * hw, y = r / g.Wi, x = r - y * g.Wi;
    const int tap = k / g.Co, co = k - tap * g.Co, ky = tap / 3, kx = tap - ky * 3;
    const int ny = y + 1 - ky, nx = x + 1 - kx;
    if (ny < 0 || nx < 0 || ny % g.stride || nx % g.stride) return 0;
    const int oy = ny / g.stride, ox = nx / g.stride;
    if (oy >= g.Ho || ox >= g.Wo) return 0;
    return f2bf(relu_mask_grad(a, ((int64_t)b * g.Ho + oy) * g.Wo + ox, co));
  } else {
    // wgrad: A[m = tap-channel k'][k = pixel] = im2col(x)[pixel][k']; row 9 Ci
    // (present when the caller sets M = 9 Ci + 1) is all ones, so that row of the
    // product is the bias gradient, the sum of the masked output gradient
    const int kk = m;
    if (kk == 9 * g.Ci) return k < g.B * g.Ho * g.Wo ? (uint16_t)0x3F80u : (uint16_t)0;
    if (kk > 9 * g.Ci) return 0;
    const int tap = kk / g.Ci, ci = kk - tap * g.Ci, ky = tap / 3, kx = tap - ky * 3;
    const int hw = g.Ho * g.Wo, b = k / hw, r = k - b * hw, oy = r / g.Wo, ox = r - oy * g.Wo;
    if (b >= g.B) return 0;
    const int iy = oy * g.stride - 1 + ky, ix = ox * g.stride - 1 + kx;
    if (iy < 0 || iy >= g.Hi || ix < 0 || ix >= g.Wi) return 0;
    return a.x[(((int64_t)b * g.Hi + iy) * g.Wi + ix) * g.Ci + ci];
  }
}

// B operand element (row k, column n).
template <int MODE>
__device__ __forceinline__ uint16_t gather_b(const ConvArgs& a, int k, int n) {
  const ConvGeom& g = a.g;
  if (MODE == CONV_FWD) {
    if (k >= 9 * g.Ci) return 0;
    return a.w[(int64_t)k * g.Co + n];
  } else if (MODE == CONV_DGRAD) {
    const int tap = k / g.Co, co = k - tap * g.Co;
    return a.w[((int64_t)tap * g.Ci + n) * g.Co + co];
  } else {
    const int hw = g.Ho * g.Wo;
    if (k >= g.B * hw) return 0;
    return f2bf(relu_mask_grad(a, k, n));
  }
}

// ---- vectorised tile loads -------------------------------------------------------
// When the channel dimension that runs along a 16-wide k step (FWD: Ci, DGRAD: Co)
// or along a group of 8 rows / columns (WGRAD: Ci and Co) is a multiple of 16 / 8,
// a step's elements are contiguous channels of one pixel and one tap: they are
// fetched 8 at a time (16 bytes) with the pixel's coordinates computed once.
__device__ __forceinline__ uint4 ld16(const uint16_t* p) { return *reinterpret_cast<const uint4*>(p); }

__device__ __forceinline__ uint4 relu_mask8(uint4 g, uint4 y) {
  // bf16 gradient kept where the bf16 activation is > 0 (the ReLU was open)
  uint32_t gv[4] = {g.x, g.y, g.z, g.w}, yv[4] = {y.x, y.y, y.z, y.w}, o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t ylo = yv[q] & 0xFFFFu, yhi = yv[q] >> 16;
    const uint32_t mlo = (ylo != 0u && !(ylo & 0x8000u)) ? 0xFFFFu : 0u;
    const uint32_t mhi = (yhi != 0u && !(yhi & 0x8000u)) ? 0xFFFF0000u : 0u;
    o[q] = gv[q] & (mlo | mhi);
  }
  return make_uint4(o[0], o[1], o[2], o[3]);
}

__device__ __forceinline__ void put8_col(uint16_t (*S)[16], int row0, int kk, uint4 v) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    S[row0 + 2 * q][kk] = (uint16_t)(w[q] & 0xFFFFu);
    S[row0 + 2 * q + 1][kk] = (uint16_t)(w[q] >> 16);
  }
}

template <int MODE, int BM>
__device__ __forceinline__ void load_a_vec(const ConvArgs& a, uint16_t (*As)[16], int m0, int k0, int kend, int t) {
  const ConvGeom& g = a.g;
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  if (MODE == CONV_FWD) {
    const int tap = k0 / g.Ci, ci0 = k0 - tap * g.Ci, ky = tap / 3, kx = tap - 3 * (tap / 3);
    for (int e = t; e < BM * 2; e += 256) {
      const int r = e >> 1, h = e & 1, m = m0 + r;
      uint4 v = z;
      if (m < a.M) {
        const int hw = g.Ho * g.Wo, b = m / hw, rr = m - b * hw, oy = rr / g.Wo, ox = rr - oy * g.Wo;
        const int iy = oy * g.stride - 1 + ky, ix = ox * g.stride - 1 + kx;
        if (iy >= 0 && iy < g.Hi && ix >= 0 && ix < g.Wi)
          v = ld16(a.x + (((int64_t)b * g.Hi + iy) * g.Wi + ix) * g.Ci + ci0 + 8 * h);
      }
      *reinterpret_cast<uint4*>(&As[r][8 * h]) = v;
    }
  } else if (MODE == CONV_DGRAD) {
    const int tap = k0 / g.Co, co0 = k0 - tap * g.Co, ky = tap / 3, kx = tap - 3 * (tap / 3);
    for (int e = t; e < BM * 2; e += 256) {
      const int r = e >> 1, h = e & 1, m = m0 + r;
      uint4 v = z;
      if (m < a.M) {
        const int hw = g.Hi * g.Wi, b = m / hw, rr = m - b * hw, y = rr / g.Wi, x = rr - y * g.Wi;
        const int ny = y + 1 - ky, nx = x + 1 - kx;
        if (ny >= 0 && nx >= 0 && ny % g.stride == 0 && nx % g.stride == 0) {
          const int oy = ny / g.stride, ox = nx / g.stride;
          if (oy < g.Ho && ox < g.Wo) {
            const int64_t at = (((int64_t)b * g.Ho + oy) * g.Wo + ox) * g.Co + co0 + 8 * h;
            v = relu_mask8(ld16(a.gy + at), ld16(a.y + at));
          }
        }
      }
      *reinterpret_cast<uint4*>(&As[r][8 * h]) = v;
    }
  } else {
    const int hw = g.Ho * g.Wo;
    for (int e = t; e < (BM / 8) * 16; e += 256) {
      const int kk = e & 15, gi = e >> 4, m = m0 + 8 * gi, k = k0 + kk;
      uint4 v = z;
      if (m == 9 * g.Ci && m < a.M && k < kend) {
        v = make_uint4(0x3F80u, 0u, 0u, 0u);  // the ones row (bias gradient), then zero rows
      } else if (m < a.M && k < kend) {
        const int tap = m / g.Ci, ci0 = m - tap * g.Ci, ky = tap / 3, kx = tap - 3 * (tap / 3);
        const int b = k / hw, rr = k - b * hw, oy = rr / g.Wo, ox = rr - oy * g.Wo;
        const int iy = oy * g.stride - 1 + ky, ix = ox * g.stride - 1 + kx;
        if (iy >= 0 && iy < g.Hi && ix >= 0 && ix < g.Wi)
          v = ld16(a.x + (((int64_t)b * g.Hi + iy) * g.Wi + ix) * g.Ci + ci0);
      }
      put8_col(As, 8 * gi, kk, v);
    }
  }
}

template <int MODE, int BN>
__device__ __forceinline__ void load_b_vec(const ConvArgs& a, uint16_t (*Bs)[16], int n0, int k0, int kend, int t) {
  const ConvGeom& g = a.g;
  const uint4 z = make_uint4(0u, 0u, 0u, 0u);
  if (MODE == CONV_FWD) {
    for (int e = t; e < (BN / 8) * 16; e += 256) {
      const int kk = e / (BN / 8), c = e - kk * (BN / 8), n = n0 + 8 * c;
      const uint4 v = (n < a.N && k0 + kk < kend) ? ld16(a.w + (int64_t)(k0 + kk) * g.Co + n) : z;
      put8_col(Bs, 8 * c, kk, v);
    }
  } else if (MODE == CONV_DGRAD) {
    const int tap = k0 / g.Co, co0 = k0 - tap * g.Co;
    for (int e = t; e < BN * 2; e += 256) {
      const int c = e >> 1, h = e & 1, n = n0 + c;
      const uint4 v = n < a.N ? ld16(a.w + ((int64_t)tap * g.Ci + n) * g.Co + co0 + 8 * h) : z;
      *reinterpret_cast<uint4*>(&Bs[c][8 * h]) = v;
    }
  } else {
    for (int e = t; e < (BN / 8) * 16; e += 256) {
      const int kk = e & 15, c = e >> 4, n = n0 + 8 * c, k = k0 + kk;
      uint4 v = z;
      if (n < a.N && k < kend) {
        const int64_t at = (int64_t)k * g.Co + n;
        v = relu_mask8(ld16(a.gy + at), ld16(a.y + at));
      }
      put8_col(Bs, 8 * c, kk, v);
    }
  }
}

// One workgroup computes a BM x BN tile of C with 4 waves (2 x 2), each wave a
// (BM/2) x (BN/2) block of 16 x 16 MFMA tiles.  K advances 32 at a time, as two
// LDS sub-tiles of 16 stored [sub][row][16], so every MFMA operand is one 16-byte
// LDS read: A lane l reads row l%16 of sub-tile l/32, k 8((l/16)%2)..+7; B lane l
// reads column l%16 likewise (A and B agree on which k each lane holds, which is
// all the product needs); C lane l holds rows 4(l/16)..+3 of column l%16
// (v_mfma_f32_16x16x32_bf16, gfx950's BF16 shape with 32 products per lane group).
template <int MODE, int BM, int BN, bool VA, bool VB>
__global__ void __launch_bounds__(256) k_conv_gemm(ConvArgs a) {
  constexpr int WM = BM / 2, WN = BN / 2, TM = WM / 16, TN = WN / 16;
  __shared__ __align__(16) uint16_t As[2][BM][16];
  __shared__ __align__(16) uint16_t Bs[2][BN][16];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
  int kbeg = 0, kend = a.K;
  if (MODE == CONV_WGRAD) {
    kbeg = blockIdx.z * a.k_chunk;
    kend = min(a.K, kbeg + a.k_chunk);
  }
  f32x4 acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int sub = lane >> 5, kq = 8 * ((lane >> 4) & 1);
  for (int k0 = kbeg; k0 < kend; k0 += 32) {
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int ks = k0 + 16 * s;
      if (ks >= kend) {  // (workgroup-uniform) past the end: a zero sub-tile
        for (int e = t; e < BM * 16; e += 256) As[s][e >> 4][e & 15] = 0;
        for (int e = t; e < BN * 16; e += 256) Bs[s][e >> 4][e & 15] = 0;
        continue;
      }
      if constexpr (VA) {
        load_a_vec<MODE, BM>(a, As[s], m0, ks, kend, t);
      } else {
        for (int e = t; e < BM * 16; e += 256) {
          const int r = e >> 4, kk = e & 15, m = m0 + r, k = ks + kk;
          As[s][r][kk] = (m < a.M && k < kend) ? gather_a<MODE>(a, m, k) : (uint16_t)0;
        }
      }
      if constexpr (VB) {
        load_b_vec<MODE, BN>(a, Bs[s], n0, ks, kend, t);
      } else {
        for (int e = t; e < BN * 16; e += 256) {
          const int c = e >> 4, kk = e & 15, n = n0 + c, k = ks + kk;
          Bs[s][c][kk] = (n < a.N && k < kend) ? gather_b<MODE>(a, k, n) : (uint16_t)0;
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < TM; ++i) {
      const bf16x8 av = *reinterpret_cast<const bf16x8*>(&As[sub][wm * WM + i * 16 + (lane & 15)][kq]);
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&Bs[sub][wn * WN + j * 16 + (lane & 15)][kq]);
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  // epilogue
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * WM + i * 16 + 4 * (lane >> 4) + r;
        const int n = n0 + wn * WN + j * 16 + (lane & 15);
        if (m >= a.M || n >= a.N) continue;
        const float v = acc[i][j][r];
        if (MODE == CONV_FWD) {
          a.out_bf16[(int64_t)m * a.N + n] = f2bf(fmaxf(v + a.bias[n], 0.0f));
        } else if (MODE == CONV_DGRAD) {
          a.out_bf16[(int64_t)m * a.N + n] = f2bf(v);
        } else {
          a.out_f32[((int64_t)blockIdx.z * a.M + m) * a.N + n] = v;
        }
      }
}

}  // namespace osog

namespace osog {

// ---- small VALU kernels ----------------------------------------------------------
// Input: x = I / 4 - 1 (BF16, one channel): the empty DIC background at bias
// pi/2 (|2i sin(theta)|^2 = 4) maps to 0; absolute brightness is kept because
// it carries the bias.
__global__ void __launch_bounds__(256) k_cnn_input(const float* __restrict__ img, int64_t n,
                                                   uint16_t* __restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] = f2bf(img[i] * 0.25f - 1.0f);
}

// Global average pool of the last activations [B][hw][C] -> p [B][C].
__global__ void __launch_bounds__(256) k_cnn_pool(const uint16_t* __restrict__ a, int hw, int C,
                                                  float* __restrict__ p) {
  const int b = blockIdx.x, c = threadIdx.x;
  if (c >= C) return;
  float s = 0.0f;
  for (int i = 0; i < hw; ++i) s += bf2f(a[((int64_t)b * hw + i) * C + c]);
  p[b * C + c] = s / (float)hw;
}

// Dense head, one 128-thread workgroup per sample:
//   h = relu(W7^T p + b7) [64], out = W8^T h + b8 [4];
//   with targets: the sample's loss term (out - t)^2 summed / (4 B), the output
//   and hidden gradients go, gh (kept per sample) and the pooled gradient gp.
__global__ void __launch_bounds__(128) k_cnn_head_fwd(const float* __restrict__ p, int B,
                                                      const float* __restrict__ W7, const float* __restrict__ b7,
                                                      const float* __restrict__ W8, const float* __restrict__ b8,
                                                      float* __restrict__ pred, const float* __restrict__ targets,
                                                      float* __restrict__ hs, float* __restrict__ gos,
                                                      float* __restrict__ ghs, float* __restrict__ gp,
                                                      float* __restrict__ loss_b) {
  __shared__ float h[64], go[4], gh[64], pp[128];
  const int t = threadIdx.x, b = blockIdx.x;
  pp[t] = p[b * 128 + t];
  __syncthreads();
  if (t < 64) {
    float s = b7[t];
    for (int i = 0; i < 128; ++i) s += W7[i * 64 + t] * pp[i];
    h[t] = fmaxf(s, 0.0f);
    hs[b * 64 + t] = h[t];
  }
  __syncthreads();
  if (t < 4) {
    float s = b8[t];
    for (int i = 0; i < 64; ++i) s += W8[i * 4 + t] * h[i];
    pred[b * 4 + t] = s;
    if (targets) {
      go[t] = 2.0f * (s - targets[b * 4 + t]) / (float)(4 * B);
      gos[b * 4 + t] = go[t];
    }
  }
  __syncthreads();
  if (!targets) return;
  if (t == 0) {
    float l = 0.0f;
    for (int k = 0; k < 4; ++k) {
      const float d = pred[b * 4 + k] - targets[b * 4 + k];
      l += d * d;
    }
    loss_b[b] = l / (float)(4 * B);
  }
  if (t < 64) {
    float s = 0.0f;
    for (int k = 0; k < 4; ++k) s += W8[t * 4 + k] * go[k];
    gh[t] = h[t] > 0.0f ? s : 0.0f;
    ghs[b * 64 + t] = gh[t];
  }
  __syncthreads();
  float s = 0.0f;
  for (int k = 0; k < 64; ++k) s += W7[t * 64 + k] * gh[k];
  gp[b * 128 + t] = s;
}

// Head parameter gradients and the loss: one thread per output, each a sum over
// the batch in sample order.
__global__ void __launch_bounds__(256) k_cnn_head_grad(const float* __restrict__ p, const float* __restrict__ hs,
                                                       const float* __restrict__ gos, const float* __restrict__ ghs,
                                                       const float* __restrict__ loss_b, int B,
                                                       float* __restrict__ gW7, float* __restrict__ gb7,
                                                       float* __restrict__ gW8, float* __restrict__ gb8,
                                                       float* __restrict__ loss) {
  const int q = blockIdx.x * 256 + threadIdx.x;
  float s = 0.0f;
  if (q < 128 * 64) {
    const int i = q / 64, j = q % 64;
    for (int b = 0; b < B; ++b) s += p[b * 128 + i] * ghs[b * 64 + j];
    gW7[q] = s;
  } else if (q < 128 * 64 + 64) {
    const int j = q - 128 * 64;
    for (int b = 0; b < B; ++b) s += ghs[b * 64 + j];
    gb7[j] = s;
  } else if (q < 128 * 64 + 64 + 256) {
    const int e = q - 128 * 64 - 64, j = e / 4, k = e % 4;
    for (int b = 0; b < B; ++b) s += hs[b * 64 + j] * gos[b * 4 + k];
    gW8[e] = s;
  } else if (q < 128 * 64 + 64 + 256 + 4) {
    const int k = q - 128 * 64 - 64 - 256;
    for (int b = 0; b < B; ++b) s += gos[b * 4 + k];
    gb8[k] = s;
  } else if (q == 128 * 64 + 64 + 256 + 4) {
    for (int b = 0; b < B; ++b) s += loss_b[b];
    *loss = s;
  }
}
constexpr int kHeadGradOutputs = 128 * 64 + 64 + 256 + 4 + 1;

// dL/d(last activations) from the pooled gradient: gy[b][i][c] = gp[b][c] / hw.
__global__ void __launch_bounds__(256) k_cnn_unpool(const float* __restrict__ gp, int B, int hw, int C,
                                                    uint16_t* __restrict__ gy) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)B * hw * C) return;
  const int c = (int)(e % C);
  const int b = (int)(e / ((int64_t)hw * C));
  gy[e] = f2bf(gp[b * C + c] / (float)hw);
}

// out[c][i] = sum over s in [c group, (c + 1) group) of part[s][i], in order of s:
// the first level of a two-level reduce over many splits (grid.y = chunks).
__global__ void __launch_bounds__(256) k_cnn_reduce_chunks(const float* __restrict__ part, int nsplit,
                                                           int group, int64_t n, float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const int k0 = (int)blockIdx.y * group, k1 = min(nsplit, k0 + group);
  float s = 0.0f;
#pragma unroll 8
  for (int k = k0; k < k1; ++k) s += part[(int64_t)k * n + i];
  out[(int64_t)blockIdx.y * n + i] = s;
}

// out[i] = sum over s of part[s][i], in order of s.
__global__ void __launch_bounds__(256) k_cnn_reduce(const float* __restrict__ part, int nsplit, int64_t n,
                                                    float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  float s = 0.0f;
#pragma unroll 8
  for (int k = 0; k < nsplit; ++k) s += part[(int64_t)k * n + i];  // loads batched, adds in order
  out[i] = s;
}

__global__ void __launch_bounds__(256) k_cnn_to_bf16(const float* __restrict__ src, int64_t n,
                                                     uint16_t* __restrict__ dst) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) dst[i] = f2bf(src[i]);
}

// Adam (Kingma & Ba 2015) with bias correction, elementwise over all parameters.
__global__ void __launch_bounds__(256) k_cnn_adam(float* __restrict__ p, float* __restrict__ m,
                                                  float* __restrict__ v, const float* __restrict__ g,
                                                  int64_t n, float lr, float b1, float b2, float eps,
                                                  float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.0f - b1) * gi;
  const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---- host --------------------------------------------------------------------------
struct CnnLayer {
  int Ci, Co, stride;
};
static const CnnLayer kLayers[6] = {{1, 32, 2}, {32, 32, 1}, {32, 64, 2}, {64, 64, 1}, {64, 128, 2}, {128, 128, 2}};
constexpr int kHead1 = 64, kOut = 4;
constexpr int64_t kSmallGrad = 4096;  // weight + bias gradients this small split their pixels finer
constexpr int kReduceGroup = 64;      // splits per first-level sum of a two-level reduce

struct CnnOffsets {
  int64_t w[6], b[6], w7, b7, w8, b8, total;
};

static CnnOffsets cnn_offsets() {
  CnnOffsets o;
  int64_t off = 0;
  for (int l = 0; l < 6; ++l) {
    o.w[l] = off;
    off += 9LL * kLayers[l].Ci * kLayers[l].Co;
    o.b[l] = off;
    off += kLayers[l].Co;
  }
  o.w7 = off; off += 128LL * kHead1;
  o.b7 = off; off += kHead1;
  o.w8 = off; off += (int64_t)kHead1 * kOut;
  o.b8 = off; off += kOut;
  o.total = off;
  return o;
}

int64_t cnn_param_count() { return cnn_offsets().total; }

struct CnnPlan {
  int B, H, W;
  int hs[7], ws[7];  // spatial size of activation l (0 = input)
  size_t x_off[7];   // activation l offsets (bf16 elements)
  size_t act_elems, ga_elems, wbf_off[6], wbf_elems, part_elems;
  int split[6];
};


static int64_t wgrad_chunk(const CnnPlan& P, int l) {
  const int64_t K = (int64_t)P.B * P.hs[l + 1] * P.ws[l + 1];
  return (K + P.split[l] - 1) / P.split[l];
}

static CnnPlan cnn_plan(int B, int H, int W) {
  CnnPlan P{};
  P.B = B; P.H = H; P.W = W;
  P.hs[0] = H; P.ws[0] = W;
  size_t off = 0;
  P.x_off[0] = 0;
  off += (size_t)B * H * W;
  for (int l = 0; l < 6; ++l) {
    P.hs[l + 1] = kLayers[l].stride == 2 ? P.hs[l] / 2 : P.hs[l];
    P.ws[l + 1] = kLayers[l].stride == 2 ? P.ws[l] / 2 : P.ws[l];
    P.x_off[l + 1] = off;
    off += (size_t)B * P.hs[l + 1] * P.ws[l + 1] * kLayers[l].Co;
  }
  P.act_elems = off;
  size_t ga = 0;
  for (int l = 0; l <= 6; ++l) {
    const int C = l == 0 ? 1 : kLayers[l - 1].Co;
    ga = std::max(ga, (size_t)B * P.hs[l] * P.ws[l] * C);
  }
  P.ga_elems = ga;
  size_t wb = 0;
  for (int l = 0; l < 6; ++l) { P.wbf_off[l] = wb; wb += 9ull * kLayers[l].Ci * kLayers[l].Co; }
  P.wbf_elems = wb;
  size_t part = 0;
  for (int l = 0; l < 6; ++l) {
    const int64_t K = (int64_t)B * P.hs[l + 1] * P.ws[l + 1];
    // split the pixel reduction so that the weight-gradient GEMM has about 2048
    // workgroups (at most 512 splits, at least 256 pixels each); a small gradient
    // (at most kSmallGrad entries: the first layer's) gets about 4096 workgroups and up
    // to 4096 splits, whose sums are then reduced in two levels
    const int M = 9 * kLayers[l].Ci + 1, N = kLayers[l].Co;  // weights and the bias row
    const int bm = N <= 32 ? 128 : 64, bn = N <= 32 ? 32 : 64;
    const int64_t tiles = (int64_t)((M + bm - 1) / bm) * ((N + bn - 1) / bn);
    const bool small = (int64_t)M * N <= kSmallGrad;
    int64_t sp = ((small ? 4096 : 2048) + tiles - 1) / tiles;
    sp = std::min<int64_t>(sp, std::max<int64_t>(1, K / 256));
    int s = (int)std::min<int64_t>(small ? 4096 : 512, std::max<int64_t>(1, sp));
    P.split[l] = s;
    const size_t level1 = small ? (size_t)((s + kReduceGroup - 1) / kReduceGroup) * M * N : 0;
    part = std::max(part, (size_t)s * M * N + level1);
  }
  P.part_elems = part;
  return P;
}

struct CnnBufs {
  uint16_t* act;      // all activations (input + 6 layers)
  uint16_t* ga0;      // gradient ping
  uint16_t* ga1;      // gradient pong
  uint16_t* wbf;      // bf16 weights
  float* part;        // split partial sums
  float* grads;       // all parameter gradients
  float* pool;        // [B][128]
  float* gpool;       // [B][128]
  float* pred;        // [B][4]
  float* loss;        // [1]
  float* hs;          // [B][64] hidden activations of the head
  float* gos;         // [B][4] output gradients
  float* ghs;         // [B][64] hidden gradients
  float* loss_b;      // [B] per-sample loss terms
  size_t total;
};

static CnnBufs cnn_carve(void* ws, const CnnPlan& P) {
  char* base = static_cast<char*>(ws);
  size_t off = 0;
  auto take = [&](size_t bytes) { void* p = base ? base + off : nullptr; off += (bytes + 255) & ~size_t(255); return p; };
  CnnBufs b;
  b.act = (uint16_t*)take(P.act_elems * 2);
  b.ga0 = (uint16_t*)take(P.ga_elems * 2);
  b.ga1 = (uint16_t*)take(P.ga_elems * 2);
  b.wbf = (uint16_t*)take(P.wbf_elems * 2);
  b.part = (float*)take(P.part_elems * 4);
  b.grads = (float*)take((size_t)cnn_param_count() * 4);
  b.pool = (float*)take((size_t)P.B * 128 * 4);
  b.gpool = (float*)take((size_t)P.B * 128 * 4);
  b.pred = (float*)take((size_t)P.B * 4 * 4);
  b.loss = (float*)take(256);
  b.hs = (float*)take((size_t)P.B * 64 * 4);
  b.gos = (float*)take((size_t)P.B * 4 * 4);
  b.ghs = (float*)take((size_t)P.B * 64 * 4);
  b.loss_b = (float*)take((size_t)P.B * 4);
  b.total = off;
  return b;
}

size_t cnn_workspace_bytes(int B, int H, int W) { return cnn_carve(nullptr, cnn_plan(B, H, W)).total; }

static unsigned blocks(int64_t n) { return (unsigned)((n + 255) / 256); }

// Vectorised loads need the channel runs described above (16-byte aligned); the
// A and B operands are decided separately.
template <int MODE>
static bool conv_vec_a(const ConvArgs& a) {
  if (MODE == CONV_FWD) return a.g.Ci % 16 == 0;
  if (MODE == CONV_DGRAD) return a.g.Co % 16 == 0;
  return a.g.Ci % 8 == 0;
}
template <int MODE>
static bool conv_vec_b(const ConvArgs& a) {
  if (MODE == CONV_FWD) return a.g.Co % 8 == 0;
  if (MODE == CONV_DGRAD) return a.g.Co % 16 == 0;
  return a.g.Co % 8 == 0;
}

template <int MODE, int BM, int BN>
static void launch_tile(const ConvArgs& a, dim3 grid, hipStream_t s) {
  const bool va = conv_vec_a<MODE>(a), vb = conv_vec_b<MODE>(a);
  if (va && vb) hipLaunchKernelGGL((k_conv_gemm<MODE, BM, BN, true, true>), grid, dim3(256), 0, s, a);
  else if (vb) hipLaunchKernelGGL((k_conv_gemm<MODE, BM, BN, false, true>), grid, dim3(256), 0, s, a);
  else if (va) hipLaunchKernelGGL((k_conv_gemm<MODE, BM, BN, true, false>), grid, dim3(256), 0, s, a);
  else hipLaunchKernelGGL((k_conv_gemm<MODE, BM, BN, false, false>), grid, dim3(256), 0, s, a);
}

template <int MODE>
static hipError_t launch_conv(const ConvArgs& a, hipStream_t s) {
  const int kz = MODE == CONV_WGRAD ? (a.K + a.k_chunk - 1) / a.k_chunk : 1;
  if (a.N <= 32) launch_tile<MODE, 128, 32>(a, dim3((a.M + 127) / 128, (a.N + 31) / 32, kz), s);
  else launch_tile<MODE, 64, 64>(a, dim3((a.M + 63) / 64, (a.N + 63) / 64, kz), s);
  return hipGetLastError();
}

static ConvArgs conv_args(const CnnPlan& P, int l) {
  ConvArgs a{};
  a.g.B = P.B;
  a.g.Hi = P.hs[l]; a.g.Wi = P.ws[l]; a.g.Ci = kLayers[l].Ci;
  a.g.Ho = P.hs[l + 1]; a.g.Wo = P.ws[l + 1]; a.g.Co = kLayers[l].Co;
  a.g.stride = kLayers[l].stride;
  return a;
}

// Forward through the convolutions, pool and head.  targets != null: also loss and
// every gradient (into b.grads).
static hipError_t cnn_run(const CnnPlan& P, const CnnBufs& b, const float* images, const float* params,
                          const float* targets, hipStream_t s) {
  const CnnOffsets O = cnn_offsets();
  const int64_t nin = (int64_t)P.B * P.H * P.W;
  hipLaunchKernelGGL(k_cnn_input, dim3(blocks(nin)), dim3(256), 0, s, images, nin, b.act + P.x_off[0]);
  for (int l = 0; l < 6; ++l) {
    const int64_t nw = 9LL * kLayers[l].Ci * kLayers[l].Co;
    hipLaunchKernelGGL(k_cnn_to_bf16, dim3(blocks(nw)), dim3(256), 0, s, params + O.w[l], nw, b.wbf + P.wbf_off[l]);
  }
  for (int l = 0; l < 6; ++l) {
    ConvArgs a = conv_args(P, l);
    a.x = b.act + P.x_off[l];
    a.w = b.wbf + P.wbf_off[l];
    a.bias = params + O.b[l];
    a.out_bf16 = b.act + P.x_off[l + 1];
    a.M = P.B * P.hs[l + 1] * P.ws[l + 1];
    a.N = kLayers[l].Co;
    a.K = 9 * kLayers[l].Ci;
    hipError_t e = launch_conv<CONV_FWD>(a, s);
    if (e != hipSuccess) return e;
  }
  const int hw6 = P.hs[6] * P.ws[6];
  hipLaunchKernelGGL(k_cnn_pool, dim3(P.B), dim3(256), 0, s, b.act + P.x_off[6], hw6, 128, b.pool);
  hipLaunchKernelGGL(k_cnn_head_fwd, dim3(P.B), dim3(128), 0, s, b.pool, P.B, params + O.w7, params + O.b7,
                     params + O.w8, params + O.b8, b.pred, targets, b.hs, b.gos, b.ghs, b.gpool, b.loss_b);
  if (targets)
    hipLaunchKernelGGL(k_cnn_head_grad, dim3((kHeadGradOutputs + 255) / 256), dim3(256), 0, s, b.pool, b.hs, b.gos,
                       b.ghs, b.loss_b, P.B, b.grads + O.w7, b.grads + O.b7, b.grads + O.w8, b.grads + O.b8, b.loss);
  if (!targets) return hipGetLastError();
  // backward through the convolutions
  uint16_t* gy = b.ga0;
  uint16_t* gx = b.ga1;
  const int64_t n6 = (int64_t)P.B * hw6 * 128;
  hipLaunchKernelGGL(k_cnn_unpool, dim3(blocks(n6)), dim3(256), 0, s, b.gpool, P.B, hw6, 128, gy);
  for (int l = 5; l >= 0; --l) {
    ConvArgs a = conv_args(P, l);
    a.x = b.act + P.x_off[l];
    a.y = b.act + P.x_off[l + 1];
    a.gy = gy;
    a.w = b.wbf + P.wbf_off[l];
    const int64_t npix = (int64_t)P.B * P.hs[l + 1] * P.ws[l + 1];
    // weight and bias gradient in one GEMM: rows 0 .. 9 Ci - 1 the weights, row 9 Ci
    // (a row of ones in the im2col operand) the bias, which the parameter layout keeps
    // right after the weights; split over pixels, reduced in order
    if (O.b[l] != O.w[l] + 9LL * kLayers[l].Ci * kLayers[l].Co) return hipErrorInvalidValue;
    a.out_f32 = b.part;
    a.M = 9 * kLayers[l].Ci + 1;
    a.N = kLayers[l].Co;
    a.K = (int)npix;
    a.k_chunk = (int)((wgrad_chunk(P, l) + 31) / 32 * 32);  // whole 32-wide k steps
    const int nsplit = (a.K + a.k_chunk - 1) / a.k_chunk;
    hipError_t e = launch_conv<CONV_WGRAD>(a, s);
    if (e != hipSuccess) return e;
    const int64_t nw = (int64_t)a.M * a.N;
    if (nw <= kSmallGrad && nsplit > kReduceGroup) {  // two levels: chunks of kReduceGroup splits, then the chunks
      const int chunks = (nsplit + kReduceGroup - 1) / kReduceGroup;
      float* level1 = b.part + (int64_t)nsplit * nw;
      hipLaunchKernelGGL(k_cnn_reduce_chunks, dim3(blocks(nw), chunks), dim3(256), 0, s, b.part, nsplit,
                         kReduceGroup, nw, level1);
      hipLaunchKernelGGL(k_cnn_reduce, dim3(blocks(nw)), dim3(256), 0, s, level1, chunks, nw, b.grads + O.w[l]);
    } else {
      hipLaunchKernelGGL(k_cnn_reduce, dim3(blocks(nw)), dim3(256), 0, s, b.part, nsplit, nw, b.grads + O.w[l]);
    }
    if (l > 0) {  // input gradient
      ConvArgs d = a;
      d.out_bf16 = gx;
      d.M = P.B * P.hs[l] * P.ws[l];
      d.N = kLayers[l].Ci;
      d.K = 9 * kLayers[l].Co;
      d.k_chunk = 0;
      if ((e = launch_conv<CONV_DGRAD>(d, s)) != hipSuccess) return e;
      std::swap(gy, gx);
    }
  }
  return hipGetLastError();
}

hipError_t cnn_forward(int B, int H, int W, const float* images, const float* params, float* pred, void* ws,
                       hipStream_t s) {
  const CnnPlan P = cnn_plan(B, H, W);
  const CnnBufs b = cnn_carve(ws, P);
  hipError_t e = cnn_run(P, b, images, params, nullptr, s);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(pred, b.pred, sizeof(float) * B * 4, hipMemcpyDeviceToDevice, s);
}

hipError_t cnn_train_step(int B, int H, int W, const float* images, const float* targets, float* params,
                          float* m, float* v, int step, float lr, float* loss, float* grads_out, void* ws,
                          hipStream_t s) {
  const CnnPlan P = cnn_plan(B, H, W);
  const CnnBufs b = cnn_carve(ws, P);
  hipError_t e = cnn_run(P, b, images, params, targets, s);
  if (e != hipSuccess) return e;
  const int64_t n = cnn_param_count();
  if (grads_out && (e = hipMemcpyAsync(grads_out, b.grads, sizeof(float) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return e;
  if (loss && (e = hipMemcpyAsync(loss, b.loss, sizeof(float), hipMemcpyDeviceToDevice, s)) != hipSuccess) return e;
  if (step > 0) {
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
    hipLaunchKernelGGL(k_cnn_adam, dim3(blocks(n)), dim3(256), 0, s, params, m, v, b.grads, n, lr, b1, b2, 1e-8f,
                       c1, c2);
  }
  return hipGetLastError();
}

// Single convolution, for checking the MFMA kernels against a reference.
hipError_t conv3x3(int mode, int B, int Hi, int Wi, int Ci, int Co, int stride, const uint16_t* x,
                   const uint16_t* y, const uint16_t* gy, const uint16_t* w, const float* bias, uint16_t* out_bf16,
                   float* out_f32, void* ws, hipStream_t s) {
  ConvArgs a{};
  a.g.B = B; a.g.Hi = Hi; a.g.Wi = Wi; a.g.Ci = Ci; a.g.Co = Co; a.g.stride = stride;
  a.g.Ho = stride == 2 ? Hi / 2 : Hi;
  a.g.Wo = stride == 2 ? Wi / 2 : Wi;
  a.x = x; a.y = y; a.gy = gy; a.w = w; a.bias = bias;
  if (mode == CONV_FWD) {
    a.out_bf16 = out_bf16; a.M = B * a.g.Ho * a.g.Wo; a.N = Co; a.K = 9 * Ci;
    return launch_conv<CONV_FWD>(a, s);
  }
  if (mode == CONV_DGRAD) {
    a.out_bf16 = out_bf16; a.M = B * Hi * Wi; a.N = Ci; a.K = 9 * Co;
    return launch_conv<CONV_DGRAD>(a, s);
  }
  a.M = 9 * Ci; a.N = Co; a.K = B * a.g.Ho * a.g.Wo;
  const int nsplit = std::max(1, std::min(64, a.K / 4096));
  a.k_chunk = ((a.K + nsplit - 1) / nsplit + 31) / 32 * 32;
  const int ns = (a.K + a.k_chunk - 1) / a.k_chunk;
  a.out_f32 = static_cast<float*>(ws);
  hipError_t e = launch_conv<CONV_WGRAD>(a, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cnn_reduce, dim3(blocks((int64_t)a.M * a.N)), dim3(256), 0, s, a.out_f32, ns,
                     (int64_t)a.M * a.N, out_f32);
  return hipGetLastError();
}

size_t conv3x3_workspace_bytes(int mode, int B, int Hi, int Wi, int Ci, int Co, int stride) {
  if (mode != CONV_WGRAD) return 256;
  const int Ho = stride == 2 ? Hi / 2 : Hi, Wo = stride == 2 ? Wi / 2 : Wi;
  const int K = B * Ho * Wo;
  const int nsplit = std::max(1, std::min(64, K / 4096));
  const int chunk = ((K + nsplit - 1) / nsplit + 15) / 16 * 16;
  const int ns = (K + chunk - 1) / chunk;
  return (size_t)ns * 9 * Ci * Co * 4 + 256;
}

}  // namespace osog
