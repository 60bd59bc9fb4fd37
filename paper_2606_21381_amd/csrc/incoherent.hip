// Differential interference contrast as Eq. 5 writes it: the exit wave U is
// sheared by +-ds and interfered at bias theta at full resolution,
//   D(r) = U(r + ds) e^{i th} - U(r - ds) e^{-i th},   D~ = U~ S,  S = 2 i sin(2 pi f.ds + th),
// squared, and blurred by the incoherent PSF |h_obj|^2 of the objective
// (h_obj = IDFT(P), Eq. 3), scaled to unit sum:
//   I = IDFT( DFT(|D|^2) OTF ),   OTF = DFT(|h_obj|^2) / sum |h_obj|^2.
// The OTF is the pupil's normalised autocorrelation, so it vanishes for |kx|
// beyond twice the pupil's largest column: the spectrum of |D|^2 is kept on
// those columns only (the band layout of the coherent chain, with more columns).
//
// Passes 1 and 2 of the coherent chain run first with every column in band and
// the shear factor as the transfer function (their Parseval sums give the mean
// of |D|^2, which the unit-sum blur keeps: the noise scale).  Then, per call,
// since the defocus lives on the device:
//   k_inc_pupil  P on the pupil's columns, column IDFT            -> band2
//   k_inc_abs2   row IDFT, |h|^2, row DFT on the OTF's columns    -> otf (band layout)
//   k_inc_otf    column DFT, divided by sum |h|^2                 -> band2 (column-major OTF)
//   k_inc_abs2   the same on D's row spectra: |D|^2's             -> otf
//   k_inc_mul    column DFT, times the OTF, column IDFT           -> otf
//   pass 3       row IDFT on the OTF's columns, I = Re, shot noise
// All transforms are unnormalised; the scale factors are stated where applied.
#include <hip/hip_runtime.h>

#include "fft_common.h"
#include "osog_internal.h"
#include "stages.h"

namespace osog {

// element (row i, band column b) of a band of n columns, rb rows per block
__device__ __forceinline__ size_t band_at(int i, int b, int n, int rb) {
  return ((size_t)(i / rb) * n + b) * rb + (i % rb);
}

// ---- P on the pupil's columns, then its column IDFT ---------------------------
// o: the frame's optics with mode brightfield and the pupil's column range.
template <int LOGH>
__global__ void __launch_bounds__(kThreads) k_inc_pupil(OpticsArgs o, const float* __restrict__ globals,
                                                        float2* __restrict__ out, const float2* __restrict__ tw) {
  constexpr int H = 1 << LOGH;
  __shared__ float2 buf[fft_lds_f2(H)];
  __shared__ int chord[2];
  const int t = threadIdx.x, b = blockIdx.x, kx = o.kx_lo + b;
  if (t == 0) band_chord(o, kx, &chord[0], &chord[1]);
  __syncthreads();
  const float dz = globals[0];
  const int lo = chord[0], hi = chord[1];
  for (int m = t; m < H; m += kThreads) {
    const int ky = m < H / 2 ? m : m - H;
    buf[m] = (ky >= lo && ky <= hi) ? transfer(o, kx, ky, dz, 0.0f, 0.0f) : make_float2(0.0f, 0.0f);
  }
  __syncthreads();
  Stages<H, 1, 1, 1, LOGH>::run(buf, tw);
  for (int i = t; i < H; i += kThreads) out[band_at(i, b, o.kx_n, o.rb)] = buf[i];
}

// ---- rows: z = IDFT_x(in), v = |z|^2 scale, row DFT of v on the out columns ----
// One workgroup per rows_per_fft_block(W) rows; psum[group] = sum of its v.
template <int LOGW>
__global__ void __launch_bounds__(kThreads) k_inc_abs2(const float2* __restrict__ in, int in_lo, int in_n,
                                                       float2* __restrict__ out, int out_lo, int out_n, int rb,
                                                       float scale, double* __restrict__ psum,
                                                       const float2* __restrict__ tw) {
  constexpr int W = 1 << LOGW, RPB = rows_per_fft_block(W);
  __shared__ __align__(16) float2 buf[fft_lds_f2(RPB * W)];
  __shared__ double red[kThreads];
  const int t = threadIdx.x, g = blockIdx.x, row0 = g * RPB;
  for (int idx = t; idx < RPB * W; idx += kThreads) buf[idx] = make_float2(0.0f, 0.0f);
  __syncthreads();
  gather_lds<4>(
      in_n * RPB,
      [&](int idx) {
        const int b = idx / RPB, r = idx - b * RPB;
        return in[band_at(row0 + r, b, in_n, rb)];
      },
      [&](int idx, float2 v) {
        const int b = idx / RPB, r = idx - b * RPB;
        buf[r * W + ((in_lo + b) & (W - 1))] = v;
      });
  __syncthreads();
  Stages<W, RPB, 1, 1, LOGW>::run(buf, tw);
  double part = 0.0;
  for (int idx = t; idx < RPB * W; idx += kThreads) {
    const float2 z = buf[idx];
    const float v = (z.x * z.x + z.y * z.y) * scale;
    buf[idx] = make_float2(v, 0.0f);
    part += (double)v;
  }
  const double ps = block_sum(part, red);  // its barriers also order buf for the stages
  if (t == 0) psum[g] = ps;
  Stages<W, RPB, -1, 1, LOGW>::run(buf, tw);
  for (int idx = t; idx < out_n * RPB; idx += kThreads) {
    const int b = idx / RPB, r = idx - b * RPB;
    out[band_at(row0 + r, b, out_n, rb)] = buf[r * W + ((out_lo + b) & (W - 1))];
  }
}

// ---- columns: the OTF = column DFT of |h|^2's row spectra / sum |h|^2 ----------
template <int LOGH>
__global__ void __launch_bounds__(kThreads) k_inc_otf(const float2* __restrict__ in, int n, int rb,
                                                      const double* __restrict__ psum, int groups,
                                                      float2* __restrict__ otf, const float2* __restrict__ tw) {
  constexpr int H = 1 << LOGH;
  __shared__ float2 buf[fft_lds_f2(H)];
  __shared__ double red[kThreads];
  const int t = threadIdx.x, b = blockIdx.x;
  gather_lds<8>(
      H, [&](int i) { return in[band_at(i, b, n, rb)]; }, [&](int i, float2 v) { buf[i] = v; });
  double s = 0.0;
  for (int k = t; k < groups; k += kThreads) s += psum[k];
  const double total = block_sum(s, red);  // its barriers also order buf for the stages
  const float inv = total > 0.0 ? (float)(1.0 / total) : 0.0f;  // an empty pupil passes nothing
  Stages<H, 1, -1, 1, LOGH>::run(buf, tw);
  for (int m = t; m < H; m += kThreads) otf[(size_t)b * H + m] = cscale(buf[m], inv);
}

// ---- columns: DFT, times the OTF, IDFT (in place in the band) -----------------
template <int LOGH>
__global__ void __launch_bounds__(kThreads) k_inc_mul(float2* __restrict__ band, int n, int rb,
                                                      const float2* __restrict__ otf,
                                                      const float2* __restrict__ tw) {
  constexpr int H = 1 << LOGH;
  __shared__ float2 buf[fft_lds_f2(H)];
  const int t = threadIdx.x, b = blockIdx.x;
  gather_lds<8>(
      H, [&](int i) { return band[band_at(i, b, n, rb)]; }, [&](int i, float2 v) { buf[i] = v; });
  __syncthreads();
  Stages<H, 1, -1, 1, LOGH>::run(buf, tw);
  gather_lds<8>(
      H, [&](int m) { return otf[(size_t)b * H + m]; }, [&](int m, float2 v) { buf[m] = cmul(buf[m], v); });
  __syncthreads();
  Stages<H, 1, 1, 1, LOGH>::run(buf, tw);
  for (int i = t; i < H; i += kThreads) band[band_at(i, b, n, rb)] = buf[i];
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

hipError_t launch_incoherent_tail(const FramePlan& p, const float* globals, FrameBufs& b, const float2* tw,
                                  float* intensity, hipStream_t s) {
  const int groups = p.H / rows_per_fft_block(p.W);
  const double hw = (double)p.H * (double)p.W;
  // two unnormalised inverse transforms leave z = HW x; |x|^2 = |z|^2 / (HW)^2
  const float scale = (float)(1.0 / (hw * hw));
  if (p.otf_n > 0) {
    if (p.pup_n > 0) {
      OpticsArgs op = optics_args(p);
      op.mode = OSOG_BRIGHTFIELD;  // the plain pupil (no tilt in this mode)
      op.kx_lo = p.pup_lo;
      op.kx_n = p.pup_n;
#define K(LG) hipLaunchKernelGGL(k_inc_pupil<LG>, dim3(p.pup_n), dim3(kThreads), 0, s, op, globals, b.band2, tw)
      OSOG_SIZE_SWITCH(p.logH, K)
#undef K
    }
#define K(LG) hipLaunchKernelGGL(k_inc_abs2<LG>, dim3(groups), dim3(kThreads), 0, s, b.band2, p.pup_lo, p.pup_n, \
                                 b.otf, p.otf_lo, p.otf_n, p.rb, scale, b.psum, tw)
    OSOG_SIZE_SWITCH(p.logW, K)
#undef K
#define K(LG) hipLaunchKernelGGL(k_inc_otf<LG>, dim3(p.otf_n), dim3(kThreads), 0, s, b.otf, p.otf_n, p.rb, b.psum, \
                                 groups, b.band2, tw)
    OSOG_SIZE_SWITCH(p.logH, K)
#undef K
    // |D|^2 from D's row spectra (all columns, left in the band by passes 1 and 2)
#define K(LG) hipLaunchKernelGGL(k_inc_abs2<LG>, dim3(groups), dim3(kThreads), 0, s, b.band, p.kx_lo, p.kx_n, \
                                 b.otf, p.otf_lo, p.otf_n, p.rb, scale, b.psum, tw)
    OSOG_SIZE_SWITCH(p.logW, K)
#undef K
#define K(LG) hipLaunchKernelGGL(k_inc_mul<LG>, dim3(p.otf_n), dim3(kThreads), 0, s, b.otf, p.otf_n, p.rb, b.band2, tw)
    OSOG_SIZE_SWITCH(p.logH, K)
#undef K
  }
  FramePlan q = p;
  q.kx_lo = p.otf_lo;
  q.kx_n = p.otf_n;
  FrameBufs bq = b;
  bq.band = b.otf;
  // the image mean (noise scale) is the mean of |D|^2: pass 2's sums over all its columns
  return launch_pass3(q, bq, tw, intensity, s, p.kx_n);
}

}  // namespace osog
