// Integer tile binning of the particle table (steps F1-F4): per-particle pixel
// box -> pair counts -> exclusive scan -> particle-major emission of (tile key,
// particle id) pairs -> stable LSD radix sort on the key -> per-tile offsets.
// The paper composes particle patches with an atomic scatter-add (Sec. III.C,
// Eq. 7); sorting the pairs instead lets every tile sum its particles in
// ascending id with no float atomics, so the canvas is bitwise reproducible.
#include <hip/hip_runtime.h>

#include "osog_internal.h"

namespace osog {

// ---- F1: prepare records, pixel boxes and pair counts -----------------------
// The box uses only exactly rounded FP32 operations with no contraction, so the
// CPU and GPU agree bit for bit:  ext = max(a,b)*1.41421366f + 1 (prism) or
// max(a,b) + 1 (ellipsoid); [floor(c - ext), floor(c + ext)] clamped to the canvas.
__device__ __forceinline__ bool pixel_box(float cx, float cy, float a, float b, float shape, int H,
                                          int W, int4* box) {
#pragma clang fp contract(off)
  if (!(a > 0.0f) || !(b > 0.0f)) return false;
  float m = fmaxf(a, b);
  float ext = (shape < 0.5f) ? (m * 1.41421366f + 1.0f) : (m + 1.0f);
  float fx0 = floorf(cx - ext), fx1 = floorf(cx + ext);
  float fy0 = floorf(cy - ext), fy1 = floorf(cy + ext);
  if (!(fx0 <= fx1) || !(fy0 <= fy1)) return false;
  if (!(fx1 >= 0.0f) || !(fy1 >= 0.0f)) return false;
  if (!(fx0 <= (float)(W - 1)) || !(fy0 <= (float)(H - 1))) return false;
  box->x = (int)fmaxf(fx0, 0.0f);
  box->y = (int)fminf(fx1, (float)(W - 1));
  box->z = (int)fmaxf(fy0, 0.0f);
  box->w = (int)fminf(fy1, (float)(H - 1));
  return true;
}

__global__ void __launch_bounds__(kThreads) k_prepare(const float* __restrict__ soa, int64_t n,
                                                      int64_t ld, int H, int W, int tile_h,
                                                      int tile_w, PRec* __restrict__ recs,
                                                      int4* __restrict__ boxes,
                                                      int* __restrict__ counts) {
  int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n) return;
  float cx = soa[0 * ld + p], cy = soa[1 * ld + p], ang = soa[2 * ld + p];
  float a = soa[3 * ld + p], b = soa[4 * ld + p], h = soa[5 * ld + p];
  float dn = soa[6 * ld + p], shape = soa[7 * ld + p];
  int4 box;
  bool ok = pixel_box(cx, cy, a, b, shape, H, W, &box);
  int cnt = 0;
  PRec r;
#pragma unroll
  for (int k = 0; k < 16; ++k) r.f[k] = 0.0f;
  if (ok) {
    int tx0 = box.x / tile_w, tx1 = box.y / tile_w, ty0 = box.z / tile_h, ty1 = box.w / tile_h;
    cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
    double cd, sd;
    sincos((double)ang, &sd, &cd);
    float c = (float)cd, s = (float)sd;
    r.f[0] = cx; r.f[1] = cy; r.f[2] = dn * h;
    r.f[4] = c; r.f[5] = s; r.f[6] = a; r.f[7] = b;
    if (shape < 0.5f) {
      r.f[3] = 0.0f;
      const float su[4] = {-1.f, 1.f, 1.f, -1.f}, sv[4] = {-1.f, -1.f, 1.f, 1.f};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        float u = su[k] * a, v = sv[k] * b;
        r.f[8 + 2 * k] = c * u - s * v;
        r.f[9 + 2 * k] = s * u + c * v;
      }
    } else {
      r.f[3] = 1.0f;
      r.f[8] = 1.0f / a; r.f[9] = 1.0f / b;
      r.f[10] = __int_as_float(__double2loint(cd)); r.f[11] = __int_as_float(__double2hiint(cd));
      r.f[12] = __int_as_float(__double2loint(sd)); r.f[13] = __int_as_float(__double2hiint(sd));
      r.f[14] = dn; r.f[15] = h;
    }
  } else {
    r.f[3] = -1.0f;
    box = make_int4(1, 0, 1, 0);
  }
  recs[p] = r;
  boxes[p] = box;
  counts[p] = cnt;
}

// ---- F2: exclusive scan of the counts (one workgroup of 1024 threads) --------
// emit_start[p] = sum_{q<p} counts[q]; emit_start[n] = total.  scal[0] = total
// clamped to the capacity, scal[1] = 1 when the total exceeds it.
__global__ void __launch_bounds__(1024) k_scan_counts(const int* __restrict__ counts, int64_t n,
                                                      int64_t cap, long long* __restrict__ emit_start,
                                                      int* __restrict__ scal) {
  __shared__ long long part[1024];
  const int t = threadIdx.x;
  const int64_t per = (n + 1023) / 1024;
  const int64_t b0 = (int64_t)t * per, b1 = min(n, b0 + per);
  long long s = 0;
  for (int64_t p = b0; p < b1; ++p) s += counts[p];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {  // Hillis-Steele inclusive scan
    long long v = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  long long run = part[t] - s;
  for (int64_t p = b0; p < b1; ++p) {
    emit_start[p] = run;
    run += counts[p];
  }
  if (t == 1023) {
    long long total = part[1023];
    emit_start[n] = total;
    scal[0] = (int)(total <= cap ? total : 0);
    scal[1] = total > cap ? 1 : 0;
  }
}

// ---- F3: emit pairs, particle-major, tiles row-major inside each particle ---
__global__ void __launch_bounds__(kThreads) k_emit(const int4* __restrict__ boxes,
                                                   const long long* __restrict__ emit_start,
                                                   int64_t n, int tile_h, int tile_w, int ntx,
                                                   const int* __restrict__ scal,
                                                   int* __restrict__ keys, int* __restrict__ vals) {
  int64_t p = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (p >= n || scal[1]) return;
  int4 box = boxes[p];
  if (box.x > box.y) return;
  int tx0 = box.x / tile_w, tx1 = box.y / tile_w, ty0 = box.z / tile_h, ty1 = box.w / tile_h;
  long long e = emit_start[p];
  for (int ty = ty0; ty <= ty1; ++ty)
    for (int tx = tx0; tx <= tx1; ++tx) {
      keys[e] = ty * ntx + tx;
      vals[e] = (int)p;
      ++e;
    }
}

// ---- F4: stable LSD radix sort on the tile key ------------------------------
// Each of kRadixBlocks workgroups owns a contiguous slice of the pair list.
// hist[d * kRadixBlocks + blk] counts digit d in slice blk; an exclusive scan of
// that digit-major array gives every (digit, slice) its output base; the
// scatter then ranks keys inside a slice in input order (ballot-matched peers
// within a wave, per-wave counts across waves), which keeps the sort stable.
__device__ __forceinline__ void slice_of(int P, int blk, int* lo, int* hi) {
  int per = (P + kRadixBlocks - 1) / kRadixBlocks;
  *lo = min(P, blk * per);
  *hi = min(P, *lo + per);
}

__global__ void __launch_bounds__(kThreads) k_radix_hist(const int* __restrict__ keys,
                                                         const int* __restrict__ scal, int shift,
                                                         int* __restrict__ hist) {
  __shared__ int h[1 << kRadixBits];
  const int t = threadIdx.x, blk = blockIdx.x;
  h[t] = 0;
  __syncthreads();
  int lo, hi;
  slice_of(scal[1] ? 0 : scal[0], blk, &lo, &hi);
  for (int q = lo + t; q < hi; q += kThreads) atomicAdd(&h[(keys[q] >> shift) & 0xFF], 1);
  __syncthreads();
  hist[t * kRadixBlocks + blk] = h[t];
}

// Exclusive scan of the 256 x 256 digit-major histogram by one 1024-thread workgroup.
__global__ void __launch_bounds__(1024) k_radix_scan(int* __restrict__ hist) {
  constexpr int N = (1 << kRadixBits) * kRadixBlocks, PER = N / 1024;
  __shared__ int part[1024];
  const int t = threadIdx.x;
  int v[PER];
  int s = 0;
#pragma unroll
  for (int k = 0; k < PER; ++k) { v[k] = hist[t * PER + k]; s += v[k]; }
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int x = (t >= off) ? part[t - off] : 0;
    __syncthreads();
    part[t] += x;
    __syncthreads();
  }
  int run = part[t] - s;
#pragma unroll
  for (int k = 0; k < PER; ++k) { hist[t * PER + k] = run; run += v[k]; }
}

__global__ void __launch_bounds__(kThreads) k_radix_scatter(const int* __restrict__ kin,
                                                            const int* __restrict__ vin,
                                                            const int* __restrict__ scal,
                                                            int shift,
                                                            const int* __restrict__ hist,
                                                            int* __restrict__ kout,
                                                            int* __restrict__ vout) {
  __shared__ int base[1 << kRadixBits];
  __shared__ int wcnt[kThreads / 64][1 << kRadixBits];
  const int t = threadIdx.x, blk = blockIdx.x, lane = t & 63, wave = t >> 6;
  base[t] = hist[t * kRadixBlocks + blk];
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) wcnt[w][t] = 0;
  __syncthreads();
  int lo, hi;
  slice_of(scal[1] ? 0 : scal[0], blk, &lo, &hi);
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int q0 = lo; q0 < hi; q0 += kThreads) {
    const int q = q0 + t;
    const bool valid = q < hi;
    int key = 0, val = 0;
    unsigned d = 0;
    if (valid) {
      key = kin[q];
      val = vin[q];
      d = (key >> shift) & 0xFF;
    }
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int bit = 0; bit < kRadixBits; ++bit) {
      bool on = (d >> bit) & 1u;
      unsigned long long m = __ballot(on);
      peers &= on ? m : ~m;
    }
    const int rank = __popcll(peers & lt);
    if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
    __syncthreads();
    if (valid) {
      int off = base[d] + rank;
      for (int w = 0; w < wave; ++w) off += wcnt[w][d];
      kout[off] = key;
      vout[off] = val;
    }
    __syncthreads();
    int tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) { tot += wcnt[w][t]; wcnt[w][t] = 0; }
    base[t] += tot;
    __syncthreads();
  }
}

// ---- tile offsets: tile_start[k] = first sorted pair with key >= k ----------
__global__ void __launch_bounds__(kThreads) k_tile_start(const int* __restrict__ keys,
                                                         const int* __restrict__ scal, int n_tiles,
                                                         int* __restrict__ tile_start) {
  int k = blockIdx.x * kThreads + threadIdx.x;
  if (k > n_tiles) return;
  int P = scal[1] ? 0 : scal[0];
  int lo = 0, hi = P;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (keys[mid] < k) lo = mid + 1; else hi = mid;
  }
  tile_start[k] = lo;
}

hipError_t launch_binning(const FramePlan& p, const float* soa, FrameBufs& b, hipStream_t s) {
  const int64_t n = p.n;
  const int gridn = (int)((n + kThreads - 1) / kThreads);
  if (n > 0)
    hipLaunchKernelGGL(k_prepare, dim3(gridn), dim3(kThreads), 0, s, soa, n, p.ld, p.H, p.W,
                       p.tile_h, p.tile_w, b.recs, b.boxes, b.counts);
  hipLaunchKernelGGL(k_scan_counts, dim3(1), dim3(1024), 0, s, b.counts, n, p.cap, b.emit_start,
                     b.scal);
  if (n > 0)
    hipLaunchKernelGGL(k_emit, dim3(gridn), dim3(kThreads), 0, s, b.boxes, b.emit_start, n,
                       p.tile_h, p.tile_w, p.ntx, b.scal, b.keys_a, b.vals_a);
  int* kin = b.keys_a; int* vin = b.vals_a; int* kout = b.keys_b; int* vout = b.vals_b;
  for (int shift = 0; shift < p.key_bits; shift += kRadixBits) {
    hipLaunchKernelGGL(k_radix_hist, dim3(kRadixBlocks), dim3(kThreads), 0, s, kin, b.scal,
                       shift, b.hist);
    hipLaunchKernelGGL(k_radix_scan, dim3(1), dim3(1024), 0, s, b.hist);
    hipLaunchKernelGGL(k_radix_scatter, dim3(kRadixBlocks), dim3(kThreads), 0, s, kin, vin,
                       b.scal, shift, b.hist, kout, vout);
    int* tk = kin; kin = kout; kout = tk;
    int* tv = vin; vin = vout; vout = tv;
  }
  // the sorted lists end in (kin, vin); make keys_a/vals_a always hold them
  if (kin != b.keys_a) {
    b.keys_b = b.keys_a; b.vals_b = b.vals_a;
    b.keys_a = kin; b.vals_a = vin;
  }
  hipLaunchKernelGGL(k_tile_start, dim3((p.n_tiles + 1 + kThreads - 1) / kThreads),
                     dim3(kThreads), 0, s, b.keys_a, b.scal, p.n_tiles, b.tile_start);
  return hipGetLastError();
}

}  // namespace osog
