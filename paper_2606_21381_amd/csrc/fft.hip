// Wave-optics imaging chain (steps F6-F8), three LDS-staged Stockham FFT passes.
//
//   pass 1 (rows)    U = exp(i 2 pi/lambda OPD) (Eq. 2), FFT along x, keep only the
//                    kx columns the pupil can pass, store them in a blocked layout
//                    band[row block][kx][row in block]
//   pass 2 (columns) FFT along y, multiply by the transfer function H(f) of the
//                    modality (pupil and defocus, Eq. 3; DIC shear and bias, Eq. 5;
//                    oblique shift P(f + f_t)), sum |U~ H|^2 per column (Parseval:
//                    gives the image mean for the noise scale), inverse FFT along y
//   pass 3 (rows)    inverse FFT along x from the in-band columns, I = |E|^2,
//                    optional Poisson shot noise (Sec. III.C, last paragraph)
//
// Transforms are radix-8 Stockham stages (radix 4 or 2 last) on data held in
// LDS, one butterfly group per thread and a barrier between stages; twiddles
// come from a 4096-entry table built in FP64 on the host.
#include <hip/hip_runtime.h>

#include "fft_common.h"
#include "osog_internal.h"

namespace osog {

// ---------------------------------------------------------------- pass 1 -----
template <int LOGW>
__global__ void __launch_bounds__(kThreads) k_pass1(const float* __restrict__ opd, int kx_lo,
                                                    int kx_n, float phase_k,
                                                    const float2* __restrict__ tw,
                                                    float2* __restrict__ band) {
  constexpr int W = 1 << LOGW, RB = rows_per_block(W);
  __shared__ float2 buf[RB * W];
  const int t = threadIdx.x, rb = blockIdx.x;
  const float* src = opd + (size_t)rb * RB * W;
  for (int idx = t; idx < RB * W; idx += kThreads) {
    float s, c;
    sincosf(phase_k * src[idx], &s, &c);
    buf[idx] = make_float2(c, s);
  }
  __syncthreads();
  Stages<W, RB, -1, 1, LOGW>::run(buf, tw);
  float2* dst = band + (size_t)rb * kx_n * RB;
  for (int idx = t; idx < kx_n * RB; idx += kThreads) {
    const int b = idx / RB, r = idx - b * RB;
    dst[idx] = buf[r * W + ((kx_lo + b) & (W - 1))];
  }
}

// ---------------------------------------------------------------- pass 2 -----
template <int LOGH>
__global__ void __launch_bounds__(kThreads) k_pass2(float2* __restrict__ band, OpticsArgs o,
                                                    const float* __restrict__ globals,
                                                    const float2* __restrict__ tw,
                                                    double* __restrict__ colsum) {
  constexpr int H = 1 << LOGH;
  __shared__ float2 buf[H];
  __shared__ int chord[2];
  __shared__ double red[kThreads];
  const int t = threadIdx.x, b = blockIdx.x, kx = o.kx_lo + b;
  const int RB = o.rb;
  for (int i = t; i < H; i += kThreads) buf[i] = band[((size_t)(i / RB) * o.kx_n + b) * RB + (i % RB)];
  if (t == 0) band_chord(o, kx, &chord[0], &chord[1]);
  __syncthreads();
  Stages<H, 1, -1, 1, LOGH>::run(buf, tw);
  const float dz = globals[0], shear = globals[1], bias = globals[2];
  const int lo = chord[0], hi = chord[1];
  double part = 0.0;
  for (int m = t; m < H; m += kThreads) {
    const int ky = m < H / 2 ? m : m - H;
    float2 g = make_float2(0.0f, 0.0f);
    if (ky >= lo && ky <= hi) {
      g = cmul(buf[m], transfer(o, kx, ky, dz, shear, bias));
      part += (double)g.x * g.x + (double)g.y * g.y;
    }
    buf[m] = g;
  }
  red[t] = part;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) colsum[b] = red[0];
  Stages<H, 1, 1, 1, LOGH>::run(buf, tw);
  for (int i = t; i < H; i += kThreads) band[((size_t)(i / RB) * o.kx_n + b) * RB + (i % RB)] = buf[i];
}

// ---------------------------------------------------------------- pass 3 -----
template <int LOGW>
__global__ void __launch_bounds__(kThreads) k_pass3(const float2* __restrict__ band, OpticsArgs o,
                                                    const double* __restrict__ colsum,
                                                    const float2* __restrict__ tw,
                                                    float* __restrict__ out,
                                                    float* __restrict__ noise_scale) {
  constexpr int W = 1 << LOGW, RB = rows_per_block(W);
  __shared__ float2 buf[RB * W];
  __shared__ double red[kThreads];
  const int t = threadIdx.x, rb = blockIdx.x;
  for (int idx = t; idx < RB * W; idx += kThreads) buf[idx] = make_float2(0.0f, 0.0f);
  __syncthreads();
  const float2* src = band + (size_t)rb * o.kx_n * RB;
  for (int idx = t; idx < o.kx_n * RB; idx += kThreads) {
    const int b = idx / RB, r = idx - b * RB;
    buf[r * W + ((o.kx_lo + b) & (W - 1))] = src[idx];
  }
  // block 0: photon scale s = photons / mean(I), the mean from the per-column
  // Parseval sums in a fixed summation order (read by the noise kernel)
  if (o.photons > 0.0f && rb == 0) {
    double s = 0.0;
    for (int b = t; b < o.kx_n; b += kThreads) s += colsum[b];
    red[t] = s;
  }
  __syncthreads();
  if (o.photons > 0.0f && rb == 0) {
    for (int s = kThreads / 2; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    if (t == 0) {
      const double hw = (double)o.H * (double)W;
      const double mean = red[0] / (hw * hw);
      *noise_scale = mean > 0.0 ? (float)((double)o.photons / mean) : 0.0f;
    }
  }
  Stages<W, RB, 1, 1, LOGW>::run(buf, tw);
  const float inv = o.inv_hw;
  float* dst = out + (size_t)rb * RB * W;
  for (int idx = t; idx < RB * W; idx += kThreads) {
    const float2 e = buf[idx];
    const float er = e.x * inv, ei = e.y * inv;
    dst[idx] = er * er + ei * ei;
  }
}

// Shot noise in place: I <- Poisson(s I) / s, one pixel pair per thread (its
// own kernel so the sampler runs at full occupancy, not under pass 3's LDS
// budget).  The pair's shared Philox block feeds both first attempts.
__global__ void __launch_bounds__(kThreads) k_noise(float* __restrict__ img, int64_t npix,
                                                    const float* __restrict__ noise_scale,
                                                    uint32_t frame, uint32_t k0, uint32_t k1) {
  const int64_t m = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  const float scale = *noise_scale;
  if (2 * m >= npix || !(scale > 0.0f)) return;
  const float2 I = reinterpret_cast<const float2*>(img)[m];
  const uint4 r = philox4x32_10(make_uint4((uint32_t)m, frame, 0u, 0u), k0, k1);
  float2 out;
  out.x = (float)poisson(scale * I.x, r.x, r.y, (uint32_t)(2 * m), frame, k0, k1) / scale;
  out.y = (float)poisson(scale * I.y, r.z, r.w, (uint32_t)(2 * m + 1), frame, k0, k1) / scale;
  reinterpret_cast<float2*>(img)[m] = out;
}

// ------------------------------------------------------------ dispatch -------
#define OSOG_SIZE_SWITCH(LOG, CALL)                                  \
  switch (LOG) {                                                     \
    case 5: CALL(5); break;                                          \
    case 6: CALL(6); break;                                          \
    case 7: CALL(7); break;                                          \
    case 8: CALL(8); break;                                          \
    case 9: CALL(9); break;                                          \
    case 10: CALL(10); break;                                        \
    case 11: CALL(11); break;                                        \
    case 12: CALL(12); break;                                        \
    default: return hipErrorInvalidValue;                            \
  }

hipError_t launch_pass1(const FramePlan& p, const float* opd, FrameBufs& b, const float2* tw,
                        hipStream_t s) {
  const int rbn = p.H / p.rb;
#define L1(LG) hipLaunchKernelGGL(k_pass1<LG>, dim3(rbn), dim3(kThreads), 0, s, opd, p.kx_lo, \
                                  p.kx_n, p.phase_k, tw, b.band)
  OSOG_SIZE_SWITCH(p.logW, L1)
#undef L1
  return hipGetLastError();
}

hipError_t launch_pass2(const FramePlan& p, const float* globals, FrameBufs& b, const float2* tw,
                        hipStream_t s) {
  OpticsArgs o = optics_args(p);
#define L2(LG) hipLaunchKernelGGL(k_pass2<LG>, dim3(p.kx_n), dim3(kThreads), 0, s, b.band, o, \
                                  globals, tw, b.colsum)
  OSOG_SIZE_SWITCH(p.logH, L2)
#undef L2
  return hipGetLastError();
}

hipError_t launch_pass3(const FramePlan& p, FrameBufs& b, const float2* tw, float* intensity,
                        hipStream_t s) {
  OpticsArgs o = optics_args(p);
  const int rbn = p.H / p.rb;
#define L3(LG) hipLaunchKernelGGL(k_pass3<LG>, dim3(rbn), dim3(kThreads), 0, s, b.band, o, \
                                  b.colsum, tw, intensity, (float*)(b.scal + 2))
  OSOG_SIZE_SWITCH(p.logW, L3)
#undef L3
  if (p.photons > 0.0f && p.kx_n > 0) {
    const int64_t npix = (int64_t)p.H * p.W;
    hipLaunchKernelGGL(k_noise, dim3((unsigned)((npix / 2 + kThreads - 1) / kThreads)), dim3(kThreads), 0, s,
                       intensity, npix, (const float*)(b.scal + 2), p.frame, p.seed_lo, p.seed_hi);
  }
  return hipGetLastError();
}

__global__ void k_philox(const uint32_t* __restrict__ ctr, int64_t count, uint32_t k0, uint32_t k1,
                         uint32_t* __restrict__ out) {
  int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= count) return;
  uint4 c = make_uint4(ctr[4 * q], ctr[4 * q + 1], ctr[4 * q + 2], ctr[4 * q + 3]);
  uint4 r = philox4x32_10(c, k0, k1);
  out[4 * q] = r.x; out[4 * q + 1] = r.y; out[4 * q + 2] = r.z; out[4 * q + 3] = r.w;
}

hipError_t launch_philox(const uint32_t* ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t* out,
                         hipStream_t s) {
  if (count > 0)
    hipLaunchKernelGGL(k_philox, dim3((unsigned)((count + kThreads - 1) / kThreads)), dim3(kThreads),
                       0, s, ctr, count, k0, k1, out);
  return hipGetLastError();
}

}  // namespace osog
