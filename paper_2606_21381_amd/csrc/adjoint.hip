// Adjoint of the renderer (the end-to-end gradient the paper keeps, Sec. III.C
// after Eq. 7), as hand-written kernels.  For a real loss L and the complex
// gradient convention g_z = dL/dRe z + i dL/dIm z, a complex-linear map y = M x
// has g_x = M^H g_y.  The forward chain and its adjoint, pass by pass:
//
//   pass 3   E = IDFT_x(B) / (HW), I = |E|^2      g_E = 2 g_I E;  g_B = DFT_x(g_E)/(HW) on the band
//   pass 2   U~ = DFT_y(A), G = U~ H, B = IDFT_y(G) g_G = DFT_y(g_B);  g_U~ = conj(H) g_G;
//                                                   dL/dpsi = Re sum conj(g_G) U~ dH/dpsi;
//                                                   g_A = IDFT_y(g_U~)
//   pass 1   A = band of DFT_x(U),                 g_U = IDFT_x(g_A zero-filled);
//            U = e^{-tau} e^{i phi}                  g_OPD = (2 pi/lambda) Im(conj(U) g_U)
//            (tau = 0 without absorption)            g_tau = -Re(conj(U) g_U)
//   raster   OPD = sum_p dn_p t_p,                 dL/dtheta_p = sum over p's pixels of
//            tau = sum_p dmu_p t_p                   (g_OPD dn_p + g_tau dmu_p) dt_p/dtheta_p
//
// (IDFT here is unnormalised.)  Forward intermediates are recomputed by the
// caller before these kernels run; nothing of frame size is kept between calls.
// The raster adjoint gathers, for each particle, g_OPD over the tiles its pixel
// box covers -- the transpose of the tile scatter-add -- and reduces in a fixed
// order, so gradients are bitwise reproducible.
#include <hip/hip_runtime.h>

#include "fft_common.h"
#include "geometry.h"
#include "osog_internal.h"

namespace osog {

// ---- forward pass 2 writing B out of place (A stays in band for the adjoint) --
template <int LOGH>
__global__ void __launch_bounds__(kThreads) k_pass2_keep(const float2* __restrict__ band,
                                                         float2* __restrict__ band2, OpticsArgs o,
                                                         const float* __restrict__ globals,
                                                         const float2* __restrict__ tw) {
  constexpr int H = 1 << LOGH;
  __shared__ float2 buf[fft_lds_f2(H)];
  __shared__ int chord[2];
  const int t = threadIdx.x, b = blockIdx.x, kx = o.kx_lo + b, RB = o.rb;
  gather_lds<8>(
      H, [&](int i) { return band[((size_t)(i / RB) * o.kx_n + b) * RB + (i % RB)]; },
      [&](int i, float2 v) { buf[i] = v; });
  if (t == 0) band_chord(o, kx, &chord[0], &chord[1]);
  __syncthreads();
  Stages<H, 1, -1, 1, LOGH>::run(buf, tw);
  const float dz = globals[0], shear = globals[1], bias = globals[2];
  const int lo = chord[0], hi = chord[1];
  for (int m = t; m < H; m += kThreads) {
    const int ky = m < H / 2 ? m : m - H;
    buf[m] = (ky >= lo && ky <= hi) ? cmul(buf[m], transfer(o, kx, ky, dz, shear, bias))
                                    : make_float2(0.0f, 0.0f);
  }
  __syncthreads();
  Stages<H, 1, 1, 1, LOGH>::run(buf, tw);
  for (int i = t; i < H; i += kThreads) band2[((size_t)(i / RB) * o.kx_n + b) * RB + (i % RB)] = buf[i];
}

// ---- adjoint of pass 3 (rows): g_B = DFT_x(2 g_I E) / (HW) on the band --------
template <int LOGW>
__global__ void __launch_bounds__(kThreads) k_adj_pass3(float2* __restrict__ band2, OpticsArgs o,
                                                        const float* __restrict__ grad_i,
                                                        const float2* __restrict__ tw) {
  constexpr int W = 1 << LOGW, RB = rows_per_block(W);
  __shared__ float2 buf[fft_lds_f2(RB * W)];
  const int t = threadIdx.x, rb = blockIdx.x;
  for (int idx = t; idx < RB * W; idx += kThreads) buf[idx] = make_float2(0.0f, 0.0f);
  __syncthreads();
  float2* blk = band2 + (size_t)rb * o.kx_n * RB;
  gather_lds<4>(
      o.kx_n * RB, [&](int idx) { return blk[idx]; },
      [&](int idx, float2 v) {
        const int b = idx / RB, r = idx - b * RB;
        buf[r * W + ((o.kx_lo + b) & (W - 1))] = v;
      });
  __syncthreads();
  Stages<W, RB, 1, 1, LOGW>::run(buf, tw);
  const float inv = o.inv_hw;
  const float* gi = grad_i + (size_t)rb * RB * W;
  constexpr int NP = RB * W, LB = 8;
  for (int i0 = t; i0 < NP; i0 += LB * kThreads) {
    float gv[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u)
      if (i0 + u * kThreads < NP) gv[u] = gi[i0 + u * kThreads];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int idx = i0 + u * kThreads;
      if (idx < NP) {
        const float2 e = buf[idx];
        const float g2 = 2.0f * gv[u] * inv;
        buf[idx] = make_float2(g2 * e.x * inv, g2 * e.y * inv);  // g_E / (HW), E = B~/(HW)
      }
    }
  }
  __syncthreads();
  Stages<W, RB, -1, 1, LOGW>::run(buf, tw);
  for (int idx = t; idx < o.kx_n * RB; idx += kThreads) {
    const int b = idx / RB, r = idx - b * RB;
    blk[idx] = buf[r * W + ((o.kx_lo + b) & (W - 1))];
  }
}

// ---- adjoint of pass 2 (columns) ---------------------------------------------
template <int LOGH>
__global__ void __launch_bounds__(kThreads) k_adj_pass2(const float2* __restrict__ band,
                                                        float2* __restrict__ band2, OpticsArgs o,
                                                        const float* __restrict__ globals,
                                                        const float2* __restrict__ tw,
                                                        double* __restrict__ colgrad) {
  constexpr int H = 1 << LOGH;
  __shared__ float2 ua[fft_lds_f2(H)];
  __shared__ float2 gb[fft_lds_f2(H)];
  __shared__ int chord[2];
  __shared__ double red[kThreads / 64];
  const int t = threadIdx.x, b = blockIdx.x, kx = o.kx_lo + b, RB = o.rb;
  gather_lds<4>(
      H, [&](int i) { return band[((size_t)(i / RB) * o.kx_n + b) * RB + (i % RB)]; },
      [&](int i, float2 v) { ua[i] = v; });
  gather_lds<4>(
      H, [&](int i) { return band2[((size_t)(i / RB) * o.kx_n + b) * RB + (i % RB)]; },
      [&](int i, float2 v) { gb[i] = v; });
  if (t == 0) band_chord(o, kx, &chord[0], &chord[1]);
  __syncthreads();
  Stages<H, 1, -1, 1, LOGH>::run(ua, tw);  // U~
  Stages<H, 1, -1, 1, LOGH>::run(gb, tw);  // g_G
  const float dz = globals[0], shear = globals[1], bias = globals[2];
  const int lo = chord[0], hi = chord[1];
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  for (int m = t; m < H; m += kThreads) {
    const int ky = m < H / 2 ? m : m - H;
    float2 out = make_float2(0.0f, 0.0f);
    if (ky >= lo && ky <= hi) {
      const float2 g = gb[m], u = ua[m];
      float2 ddz, dsh, dbi;
      transfer_grads(o, kx, ky, dz, shear, bias, &ddz, &dsh, &dbi);
      const float2 cgu = cmul(cconj(g), u);  // conj(g_G) U~
      p0 += (double)cmul(cgu, ddz).x;
      p1 += (double)cmul(cgu, dsh).x;
      p2 += (double)cmul(cgu, dbi).x;
      out = cmul(cconj(transfer(o, kx, ky, dz, shear, bias)), g);
    }
    gb[m] = out;
  }
  // fixed-order column sums; their barriers also order gb for the stages
  const double s0 = block_sum(p0, red), s1 = block_sum(p1, red), s2 = block_sum(p2, red);
  if (t == 0) {
    colgrad[b] = s0;
    colgrad[(size_t)o.kx_n + b] = s1;
    colgrad[2 * (size_t)o.kx_n + b] = s2;
  }
  Stages<H, 1, 1, 1, LOGH>::run(gb, tw);  // g_A
  for (int i = t; i < H; i += kThreads) band2[((size_t)(i / RB) * o.kx_n + b) * RB + (i % RB)] = gb[i];
}

// ---- adjoint of pass 1 (rows): g_OPD ------------------------------------------
// (absorbing frames: tau and gtau not null; grad_opd, if given, holds dL/dOPD
// then dL/dtau, one plane each)
template <int LOGW>
__global__ void __launch_bounds__(kThreads) k_adj_pass1(const float2* __restrict__ band2, OpticsArgs o,
                                                        const float* __restrict__ opd,
                                                        const float* __restrict__ tau,
                                                        const float* __restrict__ grad_opd,
                                                        float phase_k, float inv_lambda,
                                                        const float2* __restrict__ tw,
                                                        float* __restrict__ gopd, float* __restrict__ gtau,
                                                        int64_t plane) {
  constexpr int W = 1 << LOGW, RB = rows_per_block(W);
  __shared__ float2 buf[fft_lds_f2(RB * W)];
  const int t = threadIdx.x, rb = blockIdx.x;
  for (int idx = t; idx < RB * W; idx += kThreads) buf[idx] = make_float2(0.0f, 0.0f);
  __syncthreads();
  const float2* blk = band2 + (size_t)rb * o.kx_n * RB;
  gather_lds<4>(
      o.kx_n * RB, [&](int idx) { return blk[idx]; },
      [&](int idx, float2 v) {
        const int b = idx / RB, r = idx - b * RB;
        buf[r * W + ((o.kx_lo + b) & (W - 1))] = v;
      });
  __syncthreads();
  Stages<W, RB, 1, 1, LOGW>::run(buf, tw);  // g_U
  const size_t off = (size_t)rb * RB * W;
  constexpr int NP = RB * W, LB = 8;
  for (int i0 = t; i0 < NP; i0 += LB * kThreads) {
    float ov[LB], tv[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int idx = i0 + u * kThreads;
      if (idx < NP) {
        ov[u] = opd[off + idx];
        tv[u] = tau ? tau[off + idx] : 0.0f;
      }
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int idx = i0 + u * kThreads;
      if (idx >= NP) continue;
      float s, c;
      phase_sincos(ov[u], inv_lambda, &s, &c);
      if (tau) {  // U = e^{-tau} (c + i s), as pass 1 forms it
        const float am = expf(-tv[u]);
        c = am * c;
        s = am * s;
      }
      const float2 g = buf[idx];
      // Im(conj(U) g_U) with U = c + i s
      float go = phase_k * (c * g.y - s * g.x);
      if (grad_opd) go += grad_opd[off + idx];
      gopd[off + idx] = go;
      if (tau) {  // -Re(conj(U) g_U)
        float gt = -(c * g.x + s * g.y);
        if (grad_opd) gt += grad_opd[plane + off + idx];
        gtau[off + idx] = gt;
      }
    }
  }
}

// ---- adjoint of the rasteriser: per-particle gather over its tiles ------------
// Prism: c = dn h cov; d cov / d theta is the boundary flux of the footprint's
// velocity field through the part of its outline inside the pixel (each edge
// clipped to the pixel square by Liang-Barsky).  Ellipsoid: c = dn h sqrt(1-q)
// at the pixel centre, differentiated directly.
struct EdgeClip {
  float len, mid;  // clipped length and midpoint parameter along the edge (0..1)
};

__device__ __forceinline__ EdgeClip clip_edge(float px, float py, float qx, float qy) {
  // segment P + t (Q - P), t in [0,1], against the unit square [0,1]^2
  float t0 = 0.0f, t1 = 1.0f;
  const float dx = qx - px, dy = qy - py;
  const float pp[4] = {-dx, dx, -dy, dy};
  const float qq[4] = {px, 1.0f - px, py, 1.0f - py};
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (pp[k] == 0.0f) {
      if (qq[k] < 0.0f) return {0.0f, 0.0f};
    } else {
      const float r = qq[k] * __builtin_amdgcn_rcpf(pp[k]);
      if (pp[k] < 0.0f) t0 = fmaxf(t0, r);
      else t1 = fminf(t1, r);
    }
  }
  if (!(t1 > t0)) return {0.0f, 0.0f};
  return {(t1 - t0) * sqrtf(dx * dx + dy * dy), 0.5f * (t0 + t1)};
}

// ABS: the thickness also enters tau with weight dmu; acc[7] = dL/d dmu.
template <bool ABS>
__global__ void __launch_bounds__(kThreads) k_adj_raster(const float* __restrict__ soa, int64_t n,
                                                         int64_t ld, const PRec* __restrict__ recs,
                                                         const int4* __restrict__ boxes, int W,
                                                         int tile_h, int tile_w,
                                                         const float* __restrict__ gopd,
                                                         const float* __restrict__ gtau,
                                                         float* __restrict__ grad_soa,
                                                         const float4* __restrict__ hab_enc,
                                                         const float4* __restrict__ hab_info,
                                                         uint32_t topo_lo, uint32_t topo_hi) {
  constexpr int NA = ABS ? 8 : 7;
  // one wave per particle: its pixel box is dealt to the 64 lanes row-major
  const int lane = threadIdx.x & 63;
  // wave-uniform particle index: the record and table rows come through the scalar cache
  const int64_t p = (int64_t)blockIdx.x * (kThreads / 64) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (p >= n) return;  // the whole wave
  const PRec r = recs[p];
  const int4 box = boxes[p];
  const float h = soa[5 * ld + p], dn = soa[6 * ld + p];
  const float dmu = ABS ? soa[8 * ld + p] : 0.0f;
  float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
  if (r.f[3] >= 0.0f && box.x <= box.y) {
    // the pixels that can see the particle: prism, pixel squares meeting its footprint
    // bounds; ellipsoid or habit, pixel centres within its enlarged extents -- inside the box
    float fx0, fx1, fy0, fy1;
    if (r.f[3] == 0.0f) {
      fx0 = floorf(r.f[20]); fx1 = ceilf(r.f[21]) - 1.0f; fy0 = floorf(r.f[22]); fy1 = ceilf(r.f[23]) - 1.0f;
    } else {
      fx0 = floorf(r.f[0] - r.f[16] - 0.5f); fx1 = ceilf(r.f[0] + r.f[16] - 0.5f);
      fy0 = floorf(r.f[1] - r.f[17] - 0.5f); fy1 = ceilf(r.f[1] + r.f[17] - 0.5f);
    }
    const int x0 = (int)fmaxf(fx0, (float)box.x), x1 = (int)fminf(fx1, (float)box.y);
    const int y0 = (int)fmaxf(fy0, (float)box.z), y1 = (int)fminf(fy1, (float)box.w);
    const int bw = x1 - x0 + 1, cnt = (bw > 0 && y1 >= y0) ? bw * (y1 - y0 + 1) : 0;
    const float inv_bw = cnt > 0 ? 1.0f / (float)bw : 0.0f;
    const bool prism = r.f[3] == 0.0f;
    const float4 bb = prism ? prism_bounds(r) : make_float4(0.f, 0.f, 0.f, 0.f);
    const float c = r.f[4], s = r.f[5], a = r.f[6], b = r.f[7];
    for (int base = 0; base < cnt; base += 64) {
        const int k = base + lane;
        if (k >= cnt) continue;
        int row = (int)((float)k * inv_bw);  // then corrected to the exact quotient
        if (row * bw > k) --row;
        if ((row + 1) * bw <= k) ++row;
        const int i = y0 + row, j = x0 + (k - row * bw);
        const float g = gopd[(int64_t)i * W + j];
        const float gt = ABS ? gtau[(int64_t)i * W + j] : 0.0f;
        if (g == 0.0f && gt == 0.0f) continue;
        // dL/d(thickness) per unit thickness of this particle at this pixel
        const float gw = ABS ? g * dn + gt * dmu : g * dn;
        if (prism) {
          const float fj = (float)j, fi = (float)i;
          if (bb.y <= fj || bb.x >= fj + 1.0f || bb.w <= fi || bb.z >= fi + 1.0f) continue;
          const int cls = prism_classify(r, fj + 0.5f, fi + 0.5f, 0.0f);
          if (cls < 0) continue;
          if (cls > 0) {  // fully covered: only height, dn (and dmu) act
            acc[5] += gw;
            acc[6] += g * h;
            if (ABS) acc[7] += gt * h;
            continue;
          }
          const float cov = prism_cover(r, bb, i, j);
          acc[5] += gw * cov;
          acc[6] += g * h * cov;
          if (ABS) acc[7] += gt * h * cov;
          // corners relative to the pixel corner, CCW: (-a,-b) (a,-b) (a,b) (-a,b)
          const float X0 = fj - r.f[0], Y0 = fi - r.f[1];
          float vx[4], vy[4];
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            vx[k] = r.f[8 + 2 * k] - X0;
            vy[k] = r.f[9 + 2 * k] - Y0;
          }
          // outward normals: bottom -e_v, right e_u, top e_v, left -e_u
          const float nx[4] = {s, c, -s, -c}, ny[4] = {-c, s, c, -s};
          float fx = 0.f, fy = 0.f, fang = 0.f, fa = 0.f, fb = 0.f;
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const EdgeClip e = clip_edge(vx[k], vy[k], vx[(k + 1) & 3], vy[(k + 1) & 3]);
            if (e.len == 0.0f) continue;
            fx += nx[k] * e.len;
            fy += ny[k] * e.len;
            // local coordinate along the edge at the clipped midpoint
            if (k == 0) { fang -= e.len * (-a + 2.0f * a * e.mid); fb += e.len; }
            else if (k == 1) { fang -= e.len * (-b + 2.0f * b * e.mid); fa += e.len; }
            else if (k == 2) { fang += e.len * (a - 2.0f * a * e.mid); fb += e.len; }
            else { fang += e.len * (b - 2.0f * b * e.mid); fa += e.len; }
          }
          const float amp = ABS ? gw * h : g * r.f[2];
          acc[0] += amp * fx;
          acc[1] += amp * fy;
          acc[2] += amp * fang;
          acc[3] += amp * fa;
          acc[4] += amp * fb;
        } else if (r.f[3] == 2.0f) {
          // polyhedral habit: t = h w(U, V) (+ topography where positive), w the chord
          // between the active upper and lower faces, linear in (U, V) between creases;
          // the jump at a vertical face is not differentiated (centre sampling)
          const int k = (int)r.f[18];
          const float4 info = hab_info[k];
          const float4* enc = hab_enc + k * kMaxFaces;
          const int nf = (int)info.x;
          const float dx = ((float)j + 0.5f) - r.f[0], dy = ((float)i + 0.5f) - r.f[1];
          const float ia = r.f[8], ib = r.f[9];
          const float U = (c * dx + s * dy) * ia, V = (-s * dx + c * dy) * ib;
          float lo = -__builtin_inff(), hi = __builtin_inff(), plo = 0.f, qlo = 0.f, phi = 0.f, qhi = 0.f;
          bool ok = true;
          for (int f = 0; f < nf; ++f) {
            const float4 e = enc[f];
            const float val = e.x * U + e.y * V + e.z;
            if (e.w > 0.0f) {
              if (val < hi) { hi = val; phi = e.x; qhi = e.y; }
            } else if (e.w < 0.0f) {
              if (val > lo) { lo = val; plo = e.x; qlo = e.y; }
            } else {
              ok = ok && val <= 0.0f;
            }
          }
          if (!ok || !(hi > lo)) continue;
          const float w = hi - lo;
          float t = h * w;
          if (info.z > 0.0f) {
            t = t + info.z * value_noise((float)j + 0.5f, (float)i + 0.5f, 1.0f / info.w, (uint32_t)k, topo_lo,
                                         topo_hi);
            if (!(t > 0.0f)) continue;
          }
          acc[5] += gw * w;
          acc[6] += g * t;
          if (ABS) acc[7] += gt * t;
          const float wU = phi - plo, wV = qhi - qlo, k1 = gw * h;
          const float dUa = (-s * dx + c * dy) * ia, dVa = (-c * dx - s * dy) * ib;
          acc[0] += k1 * (wU * (-c * ia) + wV * (s * ib));
          acc[1] += k1 * (wU * (-s * ia) + wV * (-c * ib));
          acc[2] += k1 * (wU * dUa + wV * dVa);
          acc[3] += k1 * wU * (-U * ia);
          acc[4] += k1 * wV * (-V * ib);
        } else {
          const float dx = ((float)j + 0.5f) - r.f[0], dy = ((float)i + 0.5f) - r.f[1];
          const float u = c * dx + s * dy, v = -s * dx + c * dy;
          const float ia = r.f[8], ib = r.f[9];
          const float q = u * u * ia * ia + v * v * ib * ib;
          if (!(q < 1.0f)) continue;
          const float sq = sqrtf(1.0f - q);
          acc[5] += gw * sq;
          acc[6] += g * h * sq;
          if (ABS) acc[7] += gt * h * sq;
          const float dcq = -(ABS ? gw * h : g * r.f[2]) * 0.5f / fmaxf(sq, 1e-20f);  // d c / d q
          const float qu = 2.0f * u * ia * ia, qv = 2.0f * v * ib * ib;
          acc[0] += dcq * (qu * -c + qv * s);
          acc[1] += dcq * (qu * -s + qv * -c);
          acc[2] += dcq * (qu * v + qv * -u);
          acc[3] += dcq * (-2.0f * u * u * ia * ia * ia);
          acc[4] += dcq * (-2.0f * v * v * ib * ib * ib);
        }
      }
  }
  // fixed-order butterfly across the wave: bitwise reproducible
#pragma unroll
  for (int k = 0; k < NA; ++k)
    for (int off = 32; off > 0; off >>= 1) acc[k] += __shfl_xor(acc[k], off, 64);
  // rows 0-6 from acc[0..6], row 7 (shape) = 0, row 8 (dmu) = acc[7]
  if (lane < NA + 1) {
    float v = 0.0f;
#pragma unroll
    for (int k = 0; k < NA; ++k) v = (lane == k) ? acc[k] : v;
    if (lane == 7) v = 0.0f;
    if (ABS && lane == 8) v = acc[7];
    grad_soa[(int64_t)lane * ld + p] = v;
  }
}

// grad_globals[k] = sum over columns of colgrad[k][col], fixed order; [3] = 0
__global__ void __launch_bounds__(kThreads) k_adj_global(const double* __restrict__ colgrad, int kx_n,
                                                         float* __restrict__ grad_globals) {
  __shared__ double red[3][kThreads];
  const int t = threadIdx.x;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int b = t; b < kx_n; b += kThreads) {
    s0 += colgrad[b];
    s1 += colgrad[kx_n + b];
    s2 += colgrad[2 * (size_t)kx_n + b];
  }
  red[0][t] = s0;
  red[1][t] = s1;
  red[2][t] = s2;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (t < st) {
      red[0][t] += red[0][t + st];
      red[1][t] += red[1][t + st];
      red[2][t] += red[2][t + st];
    }
    __syncthreads();
  }
  if (t < 4) grad_globals[t] = t < 3 ? (float)red[t][0] : 0.0f;
}

// ------------------------------------------------------------ dispatch -------
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

hipError_t launch_pass2_keep(const FramePlan& p, const float* globals, FrameBufs& b, const float2* tw,
                             hipStream_t s) {
  OpticsArgs o = optics_args(p);
#define K(LG) hipLaunchKernelGGL(k_pass2_keep<LG>, dim3(p.kx_n), dim3(kThreads), 0, s, b.band, b.band2, o, \
                                 globals, tw)
  OSOG_SIZE_SWITCH(p.logH, K)
#undef K
  return hipGetLastError();
}

hipError_t launch_adj_pass3(const FramePlan& p, FrameBufs& b, const float2* tw, const float* grad_i,
                            hipStream_t s) {
  OpticsArgs o = optics_args(p);
#define K(LG) hipLaunchKernelGGL(k_adj_pass3<LG>, dim3(p.H / p.rb), dim3(kThreads), 0, s, b.band2, o, \
                                 grad_i, tw)
  OSOG_SIZE_SWITCH(p.logW, K)
#undef K
  return hipGetLastError();
}

hipError_t launch_adj_pass2(const FramePlan& p, const float* globals, FrameBufs& b, const float2* tw,
                            hipStream_t s) {
  OpticsArgs o = optics_args(p);
#define K(LG) hipLaunchKernelGGL(k_adj_pass2<LG>, dim3(p.kx_n), dim3(kThreads), 0, s, b.band, b.band2, o, \
                                 globals, tw, b.colgrad)
  OSOG_SIZE_SWITCH(p.logH, K)
#undef K
  return hipGetLastError();
}

hipError_t launch_adj_pass1(const FramePlan& p, const float* opd, const float* tau, const float* grad_opd,
                            FrameBufs& b, const float2* tw, hipStream_t s) {
  OpticsArgs o = optics_args(p);
  const float* ta = p.absorb ? tau : nullptr;
  const int64_t plane = (int64_t)p.H * p.W;
#define K(LG) hipLaunchKernelGGL(k_adj_pass1<LG>, dim3(p.H / p.rb), dim3(kThreads), 0, s, b.band2, o, opd, ta, \
                                 grad_opd, p.phase_k, p.inv_lambda, tw, b.gopd, b.gtau, plane)
  OSOG_SIZE_SWITCH(p.logW, K)
#undef K
  return hipGetLastError();
}

hipError_t launch_raster_adjoint(const FramePlan& p, const float* soa, FrameBufs& b, float* grad_soa,
                                 hipStream_t s) {
  const unsigned groups = (unsigned)((p.n + kThreads / 64 - 1) / (kThreads / 64));  // a wave per particle
  if (p.n > 0 && p.absorb)
    hipLaunchKernelGGL(k_adj_raster<true>, dim3(groups), dim3(kThreads), 0, s, soa, p.n, p.ld, b.recs,
                       b.boxes, p.W, p.tile_h, p.tile_w, b.gopd, b.gtau, grad_soa, p.hab_enc, p.hab_info, p.topo_lo,
                       p.topo_hi);
  else if (p.n > 0)
    hipLaunchKernelGGL(k_adj_raster<false>, dim3(groups), dim3(kThreads), 0, s, soa, p.n, p.ld, b.recs,
                       b.boxes, p.W, p.tile_h, p.tile_w, b.gopd, b.gtau, grad_soa, p.hab_enc, p.hab_info, p.topo_lo,
                       p.topo_hi);
  return hipGetLastError();
}

hipError_t launch_global_grads(const FramePlan& p, FrameBufs& b, float* grad_globals, hipStream_t s) {
  hipLaunchKernelGGL(k_adj_global, dim3(1), dim3(kThreads), 0, s, b.colgrad, p.kx_n, grad_globals);
  return hipGetLastError();
}

}  // namespace osog
