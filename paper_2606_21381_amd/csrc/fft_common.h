// Device building blocks of the imaging chain: Stockham FFT stages in LDS, the
// transfer function of each modality, the FP64 pupil-support predicate and the
// Poisson sampler.  Shared by the forward and adjoint passes.
#pragma once

#include "osog_internal.h"

namespace osog {

// Rows of the blocked band layout (and rows per adjoint row-pass workgroup): keeps
// one such workgroup's transform at 8192 points (72 KB of LDS with the stage
// padding) for W >= 1024.
__host__ __device__ constexpr int rows_per_block(int W) { return W >= 1024 ? 8192 / W : 8; }
// Rows one pass-1 / pass-3 workgroup transforms: half a band row block from
// W = 1024 up (4096 points, 36 KB of LDS with the stage padding, so four
// workgroups share a CU), else a full one.
__host__ __device__ constexpr int rows_per_fft_block(int W) { return W >= 1024 ? 4096 / W : 8; }

// Kernel-argument copy of the optics a pass needs.
struct OpticsArgs {
  int H, W, kx_lo, kx_n, rb, mode;
  int colsum_n;                     // column sums pass 3 adds for the image mean
  float inv_wdx, inv_hdx, kn, tfx, tfy, dsx_per_px, dsy_per_px, inv_hw, photons, read_sigma;
  double vx, vy, tfx_d, tfy_d, r2;  // FP64 band predicate: f = k * v, (fx+tx)^2 + (fy+ty)^2 <= r2
  uint32_t seed_lo, seed_hi, frame;
};

inline OpticsArgs optics_args(const FramePlan& p) {
  OpticsArgs o;
  o.H = p.H; o.W = p.W; o.kx_lo = p.kx_lo; o.kx_n = p.kx_n; o.rb = p.rb; o.mode = p.mode;
  o.colsum_n = p.kx_n;
  o.inv_wdx = p.inv_wdx; o.inv_hdx = p.inv_hdx; o.kn = p.kn; o.tfx = p.tfx; o.tfy = p.tfy;
  o.dsx_per_px = 0.5f * p.dx_um * p.cos_psi;  // ds = (shear/2) dx (cos psi, sin psi)
  o.dsy_per_px = 0.5f * p.dx_um * p.sin_psi;
  o.inv_hw = 1.0f / ((float)p.H * (float)p.W);
  o.photons = p.photons;
  o.read_sigma = p.read_sigma;
  o.vx = 1.0 / ((double)p.W * p.dx_d);
  o.vy = 1.0 / ((double)p.H * p.dx_d);
  o.tfx_d = p.tfx_d; o.tfy_d = p.tfy_d;
  o.r2 = p.na_over_lambda * p.na_over_lambda;
  o.seed_lo = p.seed_lo; o.seed_hi = p.seed_hi; o.frame = p.frame;
  return o;
}

// ---- small DFTs in registers; DIR = -1 forward (e^{-i...}), +1 inverse --------
template <int DIR>
__device__ __forceinline__ float2 mul_i(float2 z) {  // z * (DIR i)
  return DIR > 0 ? make_float2(-z.y, z.x) : make_float2(z.y, -z.x);
}

template <int DIR>
__device__ __forceinline__ void dft4(float2& v0, float2& v1, float2& v2, float2& v3) {
#pragma clang fp contract(off)
  float2 t0 = cadd(v0, v2), t1 = csub(v0, v2), t2 = cadd(v1, v3), t3 = mul_i<DIR>(csub(v1, v3));
  v0 = cadd(t0, t2);
  v2 = csub(t0, t2);
  v1 = cadd(t1, t3);
  v3 = csub(t1, t3);
}

template <int R, int DIR>
__device__ __forceinline__ void dft(float2* v) {
#pragma clang fp contract(off)
  if constexpr (R == 2) {
    float2 a = v[0];
    v[0] = cadd(a, v[1]);
    v[1] = csub(a, v[1]);
  } else if constexpr (R == 4) {
    dft4<DIR>(v[0], v[1], v[2], v[3]);
  } else {
    float2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    float2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<DIR>(e0, e1, e2, e3);
    dft4<DIR>(o0, o1, o2, o3);
    const float s2 = 0.70710678118654752f;
    o1 = cscale(cadd(o1, mul_i<DIR>(o1)), s2);       // * (1 + DIR i)/sqrt2
    o2 = mul_i<DIR>(o2);                              // * DIR i
    o3 = cscale(csub(mul_i<DIR>(o3), o3), s2);        // * (-1 + DIR i)/sqrt2
    v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
    v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
    v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
    v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
  }
}

// LDS bank spreading of the Stockham stages.  A stage writes its butterfly
// outputs r NS apart; with NS = 1 or 8 (radix 8) or NS = 1 or 4 (radix 4) a
// half-wave's 32 float2 stores would fall on a quarter or an eighth of the 64
// banks.  Such a stage writes point i at i + q (i / 32) instead (q = stage_pad),
// which gives each half-wave's stores 32 distinct bank pairs, and the next stage
// reads with the same q (its reads, 32 consecutive points per half-wave, stay
// spread).  The first stage reads and the last stage writes the plain layout, so
// callers never see the padding; a buffer holding n points for the stages needs
// fft_lds_f2(n) float2s.  Rows shorter than 256 points are not padded.
constexpr int kFftPadMax = 4;
__host__ __device__ constexpr int fft_lds_f2(int n) { return n + (n >> 5) * kFftPadMax; }

template <int N, int R, int NS>
__host__ __device__ constexpr int stage_pad() {
  return N < 256 ? 0 : (R == 8 ? (NS == 1 ? 1 : (NS == 8 ? 4 : 0)) : (R == 4 ? (NS == 1 ? 1 : (NS == 4 ? 4 : 0)) : 0));
}

template <int Q>
__device__ __forceinline__ int lds_at(int i) {
  return Q ? i + (i >> 5) * Q : i;
}

// Workgroup sum of one double per thread in a fixed order: an xor butterfly over
// each wave's lanes (lane 0's result is kept), then the waves' sums in wave order.
// Returns the total to every thread; `red` holds kThreads / 64 doubles of LDS and
// is free again on return.  Contains barriers: call uniformly.
__device__ __forceinline__ double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int t = threadIdx.x;
  if ((t & 63) == 0) red[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) s += red[w];
  __syncthreads();
  return s;
}

// Copy n elements load(i) -> store(i, .) for i = threadIdx.x + k kThreads with LB
// loads in flight per thread before the first is stored, so a workgroup waits on
// memory once per LB elements instead of once per element.
template <int LB, class Load, class Store>
__device__ __forceinline__ void gather_lds(int n, const Load& load, const Store& store) {
  for (int i0 = threadIdx.x; i0 < n; i0 += LB * kThreads) {
    float2 v[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int i = i0 + u * kThreads;
      if (i < n) v[u] = load(i);
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int i = i0 + u * kThreads;
      if (i < n) store(i, v[u]);
    }
  }
}

// Twiddles of the Stockham stage that follows NS transformed points with REM
// bits left (none for the first stage).  Each stage loads the next stage's
// twiddles right after its butterflies, so they arrive while the workgroup
// passes the stage's barriers and LDS writes.
template <int N, int ROWS, int NS, int REM, int MAXR>
struct StageTw {
  static constexpr int R = (REM >= 3 && MAXR == 8) ? 8 : (REM >= 2 ? 4 : 2);
  static constexpr int NB = N / R, TOT = ROWS * NB, BPT = (TOT + kThreads - 1) / kThreads;
  static constexpr bool kHas = NS > 1 && REM > 0;
  float2 w[kHas ? BPT : 1][kHas ? R : 1];
  __device__ __forceinline__ void load(const float2* __restrict__ tw) {
    if constexpr (kHas) {
      constexpr int TSTRIDE = kTwN / N;  // index r k N/(NS R) TSTRIDE < N TSTRIDE = kTwN
      const int t = threadIdx.x;
#pragma unroll
      for (int q = 0; q < BPT; ++q) {
        const int idx = t + q * kThreads;
        if (TOT % kThreads == 0 || idx < TOT) {
          const int k = (idx % NB) & (NS - 1);
#pragma unroll
          for (int r = 1; r < R; ++r) w[q][r] = tw[(r * k * (N / (NS * R))) * TSTRIDE];
        }
      }
    }
  }
};

// One Stockham autosort stage over ROWS rows of N points held in LDS, then the
// remaining stages.  NS = product of the radices done so far, REM = log2 of the
// part still to transform, MAXR = the plan's largest radix (8: radix-8 stages
// then one radix-4 or -2 stage; 4: radix-4 stages then one radix-2 stage).  Butterfly j of radix R reads x[j + r N/R],
// twiddles by W^(r (j mod NS) N/(NS R)), and writes to (j/NS) NS R + (j mod NS) + r NS.
template <int N, int ROWS, int DIR, int NS, int REM, int MAXR = 8, int QIN = 0>
struct Stages {
  using Tw = StageTw<N, ROWS, NS, REM, MAXR>;
  static __device__ __forceinline__ void run(float2* buf, const float2* __restrict__ tw) {
    Tw none;
    run(buf, tw, none);
  }
  static __device__ __forceinline__ void run(float2* buf, const float2* __restrict__ tw, const Tw& cw) {
#pragma clang fp contract(off)
    constexpr int R = Tw::R;
    constexpr int LR = R == 8 ? 3 : (R == 4 ? 2 : 1);
    constexpr int NB = N / R, TOT = ROWS * NB, BPT = (TOT + kThreads - 1) / kThreads;
    constexpr int QOUT = REM == LR ? 0 : stage_pad<N, R, NS>();
    static_assert(QIN <= kFftPadMax && QOUT <= kFftPadMax, "LDS padding beyond fft_lds_f2");
    float2 v[BPT][R];
    const int t = threadIdx.x;
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int idx = t + q * kThreads;
      if (TOT % kThreads == 0 || idx < TOT) {
        const int row = idx / NB, j = idx % NB;
#pragma unroll
        for (int r = 0; r < R; ++r) v[q][r] = buf[lds_at<QIN>(row * N + j + r * NB)];
        if constexpr (Tw::kHas) {
#pragma unroll
          for (int r = 1; r < R; ++r) {
            float2 w = cw.w[q][r];
            if (DIR < 0) w.y = -w.y;
            v[q][r] = cmul(v[q][r], w);
          }
        }
        dft<R, DIR>(v[q]);
      }
    }
    using Next = Stages<N, ROWS, DIR, NS * R, REM - LR, MAXR, QOUT>;
    typename Next::Tw nw;
    nw.load(tw);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < BPT; ++q) {
      const int idx = t + q * kThreads;
      if (TOT % kThreads == 0 || idx < TOT) {
        const int row = idx / NB, j = idx % NB;
        const int d = row * N + (j / NS) * NS * R + (j & (NS - 1));
#pragma unroll
        for (int r = 0; r < R; ++r) buf[lds_at<QOUT>(d + r * NS)] = v[q][r];
      }
    }
    __syncthreads();
    Next::run(buf, tw, nw);
  }
};

template <int N, int ROWS, int DIR, int NS, int MAXR, int QIN>
struct Stages<N, ROWS, DIR, NS, 0, MAXR, QIN> {
  using Tw = StageTw<N, ROWS, NS, 0, MAXR>;
  static __device__ __forceinline__ void run(float2*, const float2* __restrict__, const Tw&) {}
};

// ---- object field ------------------------------------------------------------
// sin and cos of the phase 2 pi opd / lambda (Eq. 2): the phase in turns, reduced
// exactly to [-1/2, 1/2] (the subtraction of the nearest integer is exact), then the
// hardware sine and cosine, which take their argument in turns.
__device__ __forceinline__ void phase_sincos(float opd, float inv_lambda, float* s, float* c) {
  const float turns = opd * inv_lambda;
  const float r = turns - __builtin_rintf(turns);
  *s = __builtin_amdgcn_sinf(r);
  *c = __builtin_amdgcn_cosf(r);
}

// ---- transfer function ------------------------------------------------------
// P(f) = exp(i dz (kz - k0)) inside the pupil (the piston exp(i dz k0) of Eq. 3 is
// dropped: it multiplies the whole field by one phase and leaves |E|^2 unchanged);
// kz - k0 = -2 pi |g|^2 / (kn + sqrt(kn^2 - |g|^2)) without cancellation, g = f + f_t.
// DIC: P (e^{i th} e^{+2 pi i f.ds} - e^{-i th} e^{-2 pi i f.ds}) = 2 i sin(2 pi f.ds + th) P.
// Incoherent DIC: the shear factor alone, 2 i sin(2 pi f.ds + th), on every bin.
__device__ __forceinline__ float2 transfer(const OpticsArgs& o, int kx, int ky, float dz,
                                           float shear, float bias) {
#pragma clang fp contract(off)
  const float two_pi = 6.283185307179586f;
  const float fx = (float)kx * o.inv_wdx, fy = (float)ky * o.inv_hdx;
  if (o.mode == OSOG_DIC_INCOHERENT) {
    const float rho = two_pi * shear * (fx * o.dsx_per_px + fy * o.dsy_per_px);
    return make_float2(0.0f, 2.0f * sinf(rho + bias));
  }
  const float gx = fx + o.tfx, gy = fy + o.tfy;
  const float g2 = gx * gx + gy * gy;
  const float kzm = -two_pi * g2 / (o.kn + sqrtf(fmaxf(o.kn * o.kn - g2, 0.0f)));
  float s, c;
  sincosf(dz * kzm, &s, &c);
  if (o.mode == OSOG_DIC) {
    const float rho = two_pi * shear * (fx * o.dsx_per_px + fy * o.dsy_per_px);
    const float sr = 2.0f * sinf(rho + bias);
    return make_float2(-sr * s, sr * c);
  }
  return make_float2(c, s);
}

// Derivatives of the transfer function with respect to (dz, shear, bias).
__device__ __forceinline__ void transfer_grads(const OpticsArgs& o, int kx, int ky, float dz,
                                               float shear, float bias, float2* d_dz,
                                               float2* d_shear, float2* d_bias) {
  const float two_pi = 6.283185307179586f;
  const float fx = (float)kx * o.inv_wdx, fy = (float)ky * o.inv_hdx;
  const float gx = fx + o.tfx, gy = fy + o.tfy;
  const float g2 = gx * gx + gy * gy;
  const float kzm = -two_pi * g2 / (o.kn + sqrtf(fmaxf(o.kn * o.kn - g2, 0.0f)));
  float s, c;
  sincosf(dz * kzm, &s, &c);
  const float2 P = make_float2(c, s);
  const float2 dP = make_float2(-kzm * s, kzm * c);  // d/dz e^{i dz kzm} = i kzm P
  if (o.mode == OSOG_DIC) {
    const float fds = fx * o.dsx_per_px + fy * o.dsy_per_px;
    const float rho = two_pi * shear * fds;
    float sn, cs;
    sincosf(rho + bias, &sn, &cs);
    // H = 2 i sin(rho + bias) P
    *d_dz = make_float2(-2.0f * sn * dP.y, 2.0f * sn * dP.x);
    const float dsh = 2.0f * cs * two_pi * fds;          // d/dshear of 2 sin(rho+bias)
    *d_shear = make_float2(-dsh * P.y, dsh * P.x);
    const float db = 2.0f * cs;
    *d_bias = make_float2(-db * P.y, db * P.x);
  } else {
    *d_dz = dP;
    *d_shear = make_float2(0.0f, 0.0f);
    *d_bias = make_float2(0.0f, 0.0f);
  }
}

// Pupil support of column kx: the signed ky range where
// (fx + tx)^2 + (fy + ty)^2 <= (NA/lambda)^2, f = k / (N dx), evaluated in FP64
// with every operation separately rounded (the same expression as the host's
// band bounds), so that no bin on the disc's edge can flip between passes.
__device__ inline void band_chord(const OpticsArgs& o, int kx, int* lo_out, int* hi_out) {
#pragma clang fp contract(off)
  if (o.mode == OSOG_DIC_INCOHERENT) {  // the shear factor has no pupil: every row
    *lo_out = -(o.H / 2);
    *hi_out = o.H / 2 - 1;
    return;
  }
  const double gx = (double)kx * o.vx + o.tfx_d;
  const double gx2 = gx * gx;
  const int kmin = -(o.H / 2), kmax = o.H / 2 - 1;
  auto pred = [&](int ky) {
    const double gy = (double)ky * o.vy + o.tfy_d;
    return gx2 + gy * gy <= o.r2;
  };
  const double cky = -o.tfy_d / o.vy;
  int c0 = (int)floor(cky);
  c0 = c0 < kmin ? kmin : (c0 > kmax ? kmax : c0);
  int c1 = c0 + 1 > kmax ? kmax : c0 + 1;
  int c;
  if (pred(c0)) c = c0;
  else if (pred(c1)) c = c1;
  else { *lo_out = 1; *hi_out = 0; return; }
  const double rem = o.r2 - gx2;
  const double hw = rem > 0.0 ? sqrt(rem) / o.vy : 0.0;
  int l = (int)fmax((double)kmin, floor(cky - hw));
  int h = (int)fmin((double)kmax, ceil(cky + hw));
  if (l > c) l = c;
  if (h < c) h = c;
  while (l < c && !pred(l)) ++l;
  while (l > kmin && pred(l - 1)) --l;
  while (h > c && !pred(h)) --h;
  while (h < kmax && pred(h + 1)) ++h;
  *lo_out = l;
  *hi_out = h;
}

// ---- Poisson sampler ---------------------------------------------------------
// Random words per frame from Philox4x32-10 (key = seed): pixels 2m and 2m+1
// share the block at counter (m, frame, 0, 0) -- words 0,1 belong to the even
// pixel, 2,3 to the odd one -- and draw any further words from their own blocks
// at counter (pixel, frame, round, 1), round = 1, 2, ...
// mean < 10: inversion by sequential search on the pixel's first word (at most
// 40 steps); mean >= 10: transformed rejection with squeeze (Hoermann 1993,
// "PTRS"), one attempt from the shared block, then two attempts per own block,
// at most 15 own blocks.  The acceptance test compares
// log(V inv_alpha / (a/us^2 + b)) with -mu + k log(mu) - log(k!), log(k!) from a
// table for k < 10 and from Stirling's series
// (x - 1/2) ln x - x + ln(2 pi)/2 + 1/(12x) - 1/(360 x^3), x = k + 1, above.
// Every operation is a separately rounded FP32 operation; square roots and
// quotients use the hardware square root and reciprocal (within 1 ulp), so a
// decision can differ from an exactly rounded evaluation only for a variate
// within an ulp or two of a threshold.
__device__ __forceinline__ float log_factorial(float k) {
#pragma clang fp contract(off)
  const float table[10] = {0.000000000e+00f, 0.000000000e+00f, 6.931471825e-01f, 1.791759491e+00f,
                           3.178053856e+00f, 4.787491798e+00f, 6.579251289e+00f, 8.525161743e+00f,
                           1.060460281e+01f, 1.280182743e+01f};
  if (k < 10.0f) return table[(int)k];
  const float x = k + 1.0f;
  const float rx = __builtin_amdgcn_rcpf(x);
  return (x - 0.5f) * logf(x) - x + 0.918938533f + rx * (1.0f / 12.0f) - (rx * rx * rx) * (1.0f / 360.0f);
}

// PTRS constants for one mean (mu >= 10).
struct PtrsConst {
  float log_mu, a, b, inv_alpha, vr;
};

__device__ __forceinline__ PtrsConst ptrs_const(float mu) {
#pragma clang fp contract(off)
  PtrsConst c;
  const float smu = __builtin_amdgcn_sqrtf(mu);  // mu >= 10: no denormal scaling needed
  c.log_mu = logf(mu);
  c.b = 0.931f + 2.53f * smu;
  c.a = -0.059f + 0.02483f * c.b;
  c.inv_alpha = 1.1239f + 1.1328f * __builtin_amdgcn_rcpf(c.b - 3.4f);
  c.vr = 0.9277f - 3.6224f * __builtin_amdgcn_rcpf(c.b - 2.0f);
  return c;
}

// The cheap part of a PTRS attempt: the candidate k and whether the squeeze
// accepts it without the log test.
__device__ __forceinline__ bool ptrs_quick(uint32_t wu, uint32_t wv, float mu, float a, float b, float vr,
                                           float* U_out, float* V_out, float* us_out, float* kf_out) {
#pragma clang fp contract(off)
  const float U = u01(wu) - 0.5f;
  const float V = u01(wv);
  const float us = 0.5f - fabsf(U);
  const float kf = floorf((((2.0f * a) * __builtin_amdgcn_rcpf(us)) + b) * U + (mu + 0.43f));
  *U_out = U; *V_out = V; *us_out = us; *kf_out = kf;
  return us >= 0.07f && V <= vr;
}

// One PTRS attempt from two words; returns k >= 0 when accepted, -1 when rejected.
__device__ __forceinline__ int ptrs_attempt(uint32_t wu, uint32_t wv, float mu, const PtrsConst& c) {
#pragma clang fp contract(off)
  float U, V, us, kf;
  if (ptrs_quick(wu, wv, mu, c.a, c.b, c.vr, &U, &V, &us, &kf)) return (int)kf;
  if (kf < 0.0f || (us < 0.013f && V > us)) return -1;
  const float lhs = logf(V * c.inv_alpha * __builtin_amdgcn_rcpf(c.a * __builtin_amdgcn_rcpf(us * us) + c.b));
  const float rhs = (-mu + kf * c.log_mu) - log_factorial(kf);
  return lhs <= rhs ? (int)kf : -1;
}

// Inversion by sequential search for mu < 10 (at most 40 steps) on one word.
__device__ __forceinline__ int poisson_small(float mu, uint32_t w0) {
#pragma clang fp contract(off)
  const float u = u01(w0);
  float p = expf(-mu);
  float F = p;
  int k = 0;
  while (u > F && k < 40) {
    ++k;
    p = p * (mu * __builtin_amdgcn_rcpf((float)k));
    F = F + p;
  }
  return k;
}

// PTRS for mu >= 10 from the pixel's two shared words, then up to 15 own blocks.
__device__ __forceinline__ int poisson_large(float mu, uint32_t w0, uint32_t w1, uint32_t pixel, uint32_t frame,
                                             uint32_t k0, uint32_t k1) {
#pragma clang fp contract(off)
  const PtrsConst c = ptrs_const(mu);
  int k = ptrs_attempt(w0, w1, mu, c);
  if (k >= 0) return k;
  for (uint32_t rnd = 1; rnd < 16; ++rnd) {
    const uint4 r = philox4x32_10(make_uint4(pixel, frame, rnd, 1u), k0, k1);
    k = ptrs_attempt(r.x, r.y, mu, c);
    if (k >= 0) return k;
    k = ptrs_attempt(r.z, r.w, mu, c);
    if (k >= 0) return k;
  }
  return (int)floorf(mu);
}

// Poisson(mu) for one pixel; (w0, w1) are its two words of the shared block.
__device__ __forceinline__ int poisson(float mu, uint32_t w0, uint32_t w1, uint32_t pixel,
                                       uint32_t frame, uint32_t k0, uint32_t k1) {
  if (!(mu > 0.0f)) return 0;
  if (mu < 10.0f) return poisson_small(mu, w0);
  return poisson_large(mu, w0, w1, pixel, frame, k0, k1);
}

}  // namespace osog
