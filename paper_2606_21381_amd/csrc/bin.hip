// Integer tile binning of the particle table (steps F1-F4): per-particle pixel
// box -> pair counts -> particle-major emission of (tile key, particle id)
// pairs -> stable two-pass LSD radix sort on the tile key -> per-tile first
// index and count.  The paper composes particle patches with an atomic
// scatter-add (Sec. III.C, Eq. 7); sorting the pairs instead lets every tile
// sum its particles in ascending id with no float atomics, so the canvas is
// bitwise reproducible.
//
// Six small kernels, none of them a single-workgroup scan:
//   k_prepare  records, boxes, counts, per-block count sums; clears the
//              counters the later kernels accumulate into
//   k_emit     each block sums the preceding blocks' totals (its emission
//              offset), scans its own counts, emits its pairs and counts their
//              low key digit per 256-pair slice
//   k_digit_offsets + k_scatter (pass 1): stable scatter on the low digit;
//              counts the high digit per output slice
//   k_digit_offsets + k_scatter (pass 2): stable scatter on the high digit;
//              marks each tile's first and one-past-last sorted index
// Integer atomics only ever form order-independent results (sums, minima).
#include <hip/hip_runtime.h>

#include "bin_common.h"
#include "osog_internal.h"

namespace osog {

// ---- F1: records, pixel boxes and pair counts --------------------------------
__global__ void __launch_bounds__(kThreads) k_prepare(const float* __restrict__ soa, int64_t n,
                                                      int64_t ld, int H, int W, int tile_h,
                                                      int tile_w, PRec* __restrict__ recs,
                                                      int4* __restrict__ boxes,
                                                      int* __restrict__ counts,
                                                      long long* __restrict__ blocksum,
                                                      int* __restrict__ clear_a, int64_t clear_a_n,
                                                      int* __restrict__ clear_b, int64_t clear_b_n,
                                                      int* __restrict__ clear_c, int64_t clear_c_n,
                                                      int* __restrict__ clear_min, int64_t clear_min_n) {
  __shared__ long long red[kThreads];
  const int t = threadIdx.x;
  const int64_t p = (int64_t)blockIdx.x * kThreads + t;
  // clear the accumulators of the later kernels (grid-stride)
  const int64_t gsz = (int64_t)gridDim.x * kThreads;
  for (int64_t q = p; q < clear_a_n; q += gsz) clear_a[q] = 0;
  for (int64_t q = p; q < clear_b_n; q += gsz) clear_b[q] = 0;
  for (int64_t q = p; q < clear_c_n; q += gsz) clear_c[q] = 0;
  for (int64_t q = p; q < clear_min_n; q += gsz) clear_min[q] = INT_MAX;
  int cnt = 0;
  if (p < n) {
    float cx = soa[0 * ld + p], cy = soa[1 * ld + p], ang = soa[2 * ld + p];
    float a = soa[3 * ld + p], b = soa[4 * ld + p], h = soa[5 * ld + p];
    float dn = soa[6 * ld + p], shape = soa[7 * ld + p];
    int4 box;
    bool ok = pixel_box(cx, cy, a, b, shape, H, W, &box);
    PRec r;
#pragma unroll
    for (int k = 0; k < 32; ++k) r.f[k] = 0.0f;
    if (ok) {
      int tx0 = box.x / tile_w, tx1 = box.y / tile_w, ty0 = box.z / tile_h, ty1 = box.w / tile_h;
      cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
      make_record(cx, cy, ang, a, b, h, dn, shape, &r);
    } else {
      r.f[3] = -1.0f;
      box = make_int4(1, 0, 1, 0);
    }
    recs[p] = r;
    boxes[p] = box;
    counts[p] = cnt;
  }
  red[t] = cnt;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) blocksum[blockIdx.x] = red[0];
}

// ---- F2/F3: offsets, emission and the first radix histogram -----------------
// hist1[d * nsl + s] = number of emitted keys with low digit d in the 256-key slice s.
// scal[0] = total pairs (0 on overflow), scal[1] = overflow flag.
__global__ void __launch_bounds__(kThreads) k_emit(const int4* __restrict__ boxes,
                                                   const int* __restrict__ counts,
                                                   const long long* __restrict__ blocksum,
                                                   int64_t n, int nblk, int64_t cap, int tile_h,
                                                   int tile_w, int ntx, int d1_bits,
                                                   long long* __restrict__ emit_start,
                                                   int* __restrict__ scal,
                                                   int* __restrict__ keys, int* __restrict__ vals,
                                                   int* __restrict__ hist1, int nsl,
                                                   int* __restrict__ tile_first,
                                                   int* __restrict__ tile_end) {
  __shared__ long long red[kThreads];
  __shared__ long long scan[kThreads];
  const int t = threadIdx.x, blk = blockIdx.x;
  // offset of this block = sum of the preceding blocks' totals; total = sum of all
  long long pre = 0, tot = 0;
  for (int b = t; b < nblk; b += kThreads) {
    const long long v = blocksum[b];
    tot += v;
    if (b < blk) pre += v;
  }
  red[t] = pre;
  scan[t] = tot;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) { red[t] += red[t + s]; scan[t] += scan[t + s]; }
    __syncthreads();
  }
  const long long base = red[0], total = scan[0];
  const bool overflow = total > cap;
  if (blk == 0 && t == 0) {
    scal[0] = overflow ? 0 : (int)total;
    scal[1] = overflow ? 1 : 0;
    emit_start[n] = total;
  }
  __syncthreads();
  // block-local exclusive scan of the counts (Hillis-Steele)
  const int64_t p = (int64_t)blk * kThreads + t;
  const int c = p < n ? counts[p] : 0;
  scan[t] = c;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    long long v = t >= off ? scan[t - off] : 0;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  long long e = base + scan[t] - c;
  if (p < n) emit_start[p] = e;
  if (!overflow && c > 0) {
    const int4 box = boxes[p];
    const int tx0 = box.x / tile_w, tx1 = box.y / tile_w, ty0 = box.z / tile_h, ty1 = box.w / tile_h;
    const int mask = (1 << d1_bits) - 1;
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) {
        const int key = ty * ntx + tx;
        keys[e] = key;
        vals[e] = (int)p;
        if (d1_bits > 0) {
          atomicAdd(&hist1[(size_t)(key & mask) * nsl + (e >> 8)], 1);
        } else {  // a single tile: the emission order is already sorted
          atomicMin(&tile_first[key], (int)e);
          atomicMax(&tile_end[key], (int)e + 1);
        }
        ++e;
      }
  }
}

// ---- F4: one stable scatter pass of the LSD radix sort ----------------------
// The pass input is cut into 256-key slices, one per workgroup.  Each slice's
// per-digit output base is (exclusive scan over digits of the digit totals) +
// (exclusive prefix of its digit over earlier slices), both from
// k_digit_offsets.  Keys are ranked inside the slice in input order (peers
// matched by ballots inside a wave, per-wave counts across waves), which keeps
// the sort stable.  The first pass counts the next digit of each key per
// output slice; the final pass marks each tile's first and last sorted index
// (only run boundaries inside a wave touch the counters).
template <bool FINAL>
__global__ void __launch_bounds__(kThreads) k_scatter(const int* __restrict__ kin,
                                                      const int* __restrict__ vin,
                                                      const int* __restrict__ scal, int nsl,
                                                      int shift, int bits,
                                                      const int* __restrict__ hist,
                                                      const int* __restrict__ dtot,
                                                      int* __restrict__ kout, int* __restrict__ vout,
                                                      int next_shift, int next_bits,
                                                      int* __restrict__ next_hist,
                                                      int* __restrict__ tile_first,
                                                      int* __restrict__ tile_end) {
  __shared__ int base[256];
  __shared__ int wcnt[kThreads / 64][256];
  const int t = threadIdx.x, blk = blockIdx.x, lane = t & 63, wave = t >> 6;
  if (scal[1]) return;
  const int P = scal[0];
  const int lo = blk * kThreads;
  if (lo >= P) return;
  const int hi = min(P, lo + kThreads);
  const int nd = 1 << bits, mask = nd - 1;
  const int tot = t < nd ? dtot[t] : 0;
  base[t] = tot;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) wcnt[w][t] = 0;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive scan of the digit totals
    int v = t >= off ? base[t - off] : 0;
    __syncthreads();
    base[t] += v;
    __syncthreads();
  }
  const int excl = (t < nd) ? base[t] - tot + hist[(size_t)t * nsl + blk] : 0;
  __syncthreads();
  base[t] = excl;
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int q = lo + t;
  const bool valid = q < hi;
  int key = 0, val = 0;
  unsigned d = 0;
  if (valid) {
    key = kin[q];
    val = vin[q];
    d = (key >> shift) & mask;
  }
  unsigned long long peers = __ballot(valid);
  for (int bit = 0; bit < bits; ++bit) {
    const bool on = (d >> bit) & 1u;
    const unsigned long long m = __ballot(on);
    peers &= on ? m : ~m;
  }
  if (!valid) peers = 0;
  const int rank = __popcll(peers & lt);
  if (valid && rank == 0) wcnt[wave][d] = __popcll(peers);
  __syncthreads();
  if (valid) {
    int off = base[d] + rank;
    for (int w = 0; w < wave; ++w) off += wcnt[w][d];
    kout[off] = key;
    vout[off] = val;
    if (FINAL) {
      // peers with one digit keep input (low-digit) order, so equal keys are
      // adjacent among them: a tile run starts/ends where the neighbouring peer differs
      const unsigned long long before = peers & lt, after = peers & ~lt & ~(1ull << lane);
      const int prev_lane = before ? 63 - __clzll(before) : -1;
      const int next_lane = after ? __ffsll(after) - 1 : -1;
      const int prev_key = __shfl(key, prev_lane < 0 ? lane : prev_lane);
      const int next_key = __shfl(key, next_lane < 0 ? lane : next_lane);
      if (prev_lane < 0 || prev_key != key) atomicMin(&tile_first[key], off);
      if (next_lane < 0 || next_key != key) atomicMax(&tile_end[key], off + 1);
    } else {
      atomicAdd(&next_hist[(size_t)((key >> next_shift) & ((1 << next_bits) - 1)) * nsl + (off >> 8)], 1);
    }
  }
}

// Per-digit exclusive prefix over slices, in place: hist[d][b] <- sum_{b'<b} hist[d][b'],
// and dtot[d] = sum over all slices.  One block per digit; each thread owns a
// contiguous run of slices.
__global__ void __launch_bounds__(kThreads) k_digit_offsets(int* __restrict__ hist, int nsl,
                                                            const int* __restrict__ scal,
                                                            int* __restrict__ dtot) {
  __shared__ int part[kThreads];
  const int t = threadIdx.x, d = blockIdx.x;
  if (scal[1]) return;
  const int nslice = (scal[0] + kThreads - 1) / kThreads;
  int* row = hist + (size_t)d * nsl;
  const int per = (nslice + kThreads - 1) / kThreads;
  const int b0 = min(nslice, t * per), b1 = min(nslice, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += row[b];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int b = b0; b < b1; ++b) {
    const int v = row[b];
    row[b] = run;
    run += v;
  }
  if (t == kThreads - 1) dtot[d] = part[t];
}

// tile_start[k] = first sorted pair with key >= k (only for the inspection API)
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
  const int nblk = (int)((n + kThreads - 1) / kThreads);
  const int gridp = nblk > 0 ? nblk : 1;
  const int d1 = (p.key_bits + 1) / 2, d2 = p.key_bits - d1;
  const int nsl = (int)((p.cap + kThreads - 1) / kThreads);  // slice capacity (row stride)
  hipLaunchKernelGGL(k_prepare, dim3(gridp), dim3(kThreads), 0, s, soa, n, p.ld, p.H, p.W, p.tile_h,
                     p.tile_w, b.recs, b.boxes, b.counts, b.blocksum, b.hist1,
                     d1 > 0 ? ((int64_t)1 << d1) * nsl : 0, b.hist2, d2 > 0 ? ((int64_t)1 << d2) * nsl : 0,
                     b.tile_end, (int64_t)p.n_tiles, b.tile_first, (int64_t)p.n_tiles);
  hipLaunchKernelGGL(k_emit, dim3(gridp), dim3(kThreads), 0, s, b.boxes, b.counts, b.blocksum, n,
                     nblk, p.cap, p.tile_h, p.tile_w, p.ntx, d1, b.emit_start, b.scal, b.keys_a,
                     b.vals_a, b.hist1, nsl, b.tile_first, b.tile_end);
  b.sorted_keys = b.keys_a;
  b.sorted_vals = b.vals_a;
  if (d1 > 0 && nblk > 0) {
    hipLaunchKernelGGL(k_digit_offsets, dim3(1 << d1), dim3(kThreads), 0, s, b.hist1, nsl, b.scal, b.dtot);
    if (d2 > 0) {
      hipLaunchKernelGGL(k_scatter<false>, dim3(nsl), dim3(kThreads), 0, s, b.keys_a, b.vals_a, b.scal,
                         nsl, 0, d1, b.hist1, b.dtot, b.keys_b, b.vals_b, d1, d2, b.hist2,
                         b.tile_first, b.tile_end);
      hipLaunchKernelGGL(k_digit_offsets, dim3(1 << d2), dim3(kThreads), 0, s, b.hist2, nsl, b.scal,
                         b.dtot + 256);
      hipLaunchKernelGGL(k_scatter<true>, dim3(nsl), dim3(kThreads), 0, s, b.keys_b, b.vals_b, b.scal,
                         nsl, d1, d2, b.hist2, b.dtot + 256, b.keys_a, b.vals_a, 0, 0, (int*)nullptr,
                         b.tile_first, b.tile_end);
    } else {
      hipLaunchKernelGGL(k_scatter<true>, dim3(nsl), dim3(kThreads), 0, s, b.keys_a, b.vals_a, b.scal,
                         nsl, 0, d1, b.hist1, b.dtot, b.keys_b, b.vals_b, 0, 0, (int*)nullptr,
                         b.tile_first, b.tile_end);
      b.sorted_keys = b.keys_b;
      b.sorted_vals = b.vals_b;
    }
  }
  return hipGetLastError();
}

hipError_t launch_tile_start(const FramePlan& p, FrameBufs& b, int* tile_start, hipStream_t s) {
  hipLaunchKernelGGL(k_tile_start, dim3((p.n_tiles + 1 + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     s, b.sorted_keys, b.scal, p.n_tiles, tile_start);
  return hipGetLastError();
}

}  // namespace osog
