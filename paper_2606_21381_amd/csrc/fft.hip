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
//                    optional Poisson shot noise (Sec. III.C, last paragraph),
//                    sampled in place on the rows the workgroup holds
//
// Transforms are radix-8 Stockham stages (radix 4 or 2 last) on data held in
// LDS, one butterfly group per thread and a barrier between stages; twiddles
// come from a 4096-entry table built in FP64 on the host.
#include <hip/hip_runtime.h>

#include "fft_common.h"
#include "osog_internal.h"
#include "stages.h"

namespace osog {

// Workgroups of consecutive row groups fill the two halves of the same band
// pieces, so each XCD (workgroup i runs on XCD i mod 8) takes one contiguous run
// of row groups and the halves meet in one L2.  per_xcd * 8 >= groups.
template <int LOGW, int MAXR>
__global__ void __launch_bounds__(kThreads) k_pass1(FrameDev F, const float2* __restrict__ tw, int per_xcd) {
  __shared__ __align__(16) char lds[fft_lds_f2(rows_per_fft_block(1 << LOGW) * (1 << LOGW)) * sizeof(float2)];
  const int g = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (g * rows_per_fft_block(1 << LOGW) < F.H) pass1_body<LOGW, MAXR>(F, g, tw, lds);
}

// Column b of the band lives in 32-byte pieces (RB rows) next to columns b +- 1,
// so neighbouring columns share cache lines: each XCD (workgroup i runs on XCD
// i mod 8) takes one contiguous run of columns, and a line is fetched once.
template <int LOGH, int MAXR>
__global__ void __launch_bounds__(kThreads) k_pass2(FrameDev F, const float2* __restrict__ tw, int per_xcd) {
  __shared__ __align__(16) char lds[fft_lds_f2(1 << LOGH) * sizeof(float2) + kThreads * sizeof(double) + 16];
  const int b = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (b < F.o.kx_n) pass2_body<LOGH, MAXR>(F, b, tw, lds);
}

template <int LOGW, int MAXR>
__global__ void __launch_bounds__(kThreads) k_pass3(FrameDev F, const float2* __restrict__ tw, int per_xcd) {
  __shared__ __align__(16) char lds[pass3_buf_bytes(1 << LOGW) + kThreads * sizeof(double)];
  const int g = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (g * rows_per_fft_block(1 << LOGW) < F.H) pass3_body<LOGW, MAXR>(F, g, tw, lds);
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

hipError_t launch_pass1(const FramePlan& p, const float* opd, const float* tau, FrameBufs& b, const float2* tw,
                        hipStream_t s) {
  FrameDev F = make_dev(p, b);
  F.opd = const_cast<float*>(opd);
  F.tau = const_cast<float*>(tau);
  const int rbn = p.H / rows_per_fft_block(p.W), per = (rbn + kXcds - 1) / kXcds;
#define L1(LG)                                                                              \
  if (p.fft_radix == 4) hipLaunchKernelGGL((k_pass1<LG, 4>), dim3(per * kXcds), dim3(kThreads), 0, s, F, tw, per); \
  else hipLaunchKernelGGL((k_pass1<LG, 8>), dim3(per * kXcds), dim3(kThreads), 0, s, F, tw, per)
  OSOG_SIZE_SWITCH(p.logW, L1)
#undef L1
  return hipGetLastError();
}

hipError_t launch_pass2(const FramePlan& p, const float* globals, FrameBufs& b, const float2* tw,
                        hipStream_t s, const float2* band_in, int in_kx_lo, int in_kx_n) {
  FrameDev F = make_dev(p, b);
  F.globals = globals;
  if (band_in) {
    F.band_in = band_in;
    F.in_kx_lo = in_kx_lo;
    F.in_kx_n = in_kx_n;
  }
  const int per = (p.kx_n + kXcds - 1) / kXcds;
#define L2(LG)                                                                                  \
  if (p.fft_radix == 4) hipLaunchKernelGGL((k_pass2<LG, 4>), dim3(per * kXcds), dim3(kThreads), 0, s, F, tw, per); \
  else hipLaunchKernelGGL((k_pass2<LG, 8>), dim3(per * kXcds), dim3(kThreads), 0, s, F, tw, per)
  OSOG_SIZE_SWITCH(p.logH, L2)
#undef L2
  return hipGetLastError();
}

hipError_t launch_pass3(const FramePlan& p, FrameBufs& b, const float2* tw, float* intensity,
                        hipStream_t s, int colsum_n) {
  FrameDev F = make_dev(p, b);
  F.intensity = intensity;
  if (colsum_n >= 0) F.o.colsum_n = colsum_n;
  const int rbn = p.H / rows_per_fft_block(p.W), per = (rbn + kXcds - 1) / kXcds;
#define L3(LG)                                                                              \
  if (p.fft_radix == 4) hipLaunchKernelGGL((k_pass3<LG, 4>), dim3(per * kXcds), dim3(kThreads), 0, s, F, tw, per); \
  else hipLaunchKernelGGL((k_pass3<LG, 8>), dim3(per * kXcds), dim3(kThreads), 0, s, F, tw, per)
  OSOG_SIZE_SWITCH(p.logW, L3)
#undef L3
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
