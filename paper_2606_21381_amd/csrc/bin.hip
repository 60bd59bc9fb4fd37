// Integer tile binning of the particle table (steps F1-F4): a one-digit
// counting sort of (tile key, particle id) pairs on the tile key, whose radix
// is the number of tiles, into fixed-size per-tile buckets.  The paper composes
// particle patches with an atomic scatter-add (Sec. III.C, Eq. 7); grouping the
// pairs by tile instead lets every tile sum its particles in ascending id with no
// float atomics, so the canvas is bitwise reproducible.
//
//   k_bin_clear  tile counters and flags = 0
//   k_bin        records, boxes, pairs per particle; every pair takes the next
//                slot of its tile's bucket through an atomic cursor
// Integer atomics only form order-independent results (counts) or slots inside
// a tile's bucket; the order of ids inside a bucket is restored by the reader,
// which sorts it (raster_tile; k_sort_segments for the inspection API).  A tile
// whose bucket overflows is read by an id-ordered scan of all particles.
#include <hip/hip_runtime.h>

#include "osog_internal.h"
#include "stages.h"

namespace osog {

__global__ void __launch_bounds__(kThreads) k_bin_clear(FrameDev F) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t < F.n_tiles) F.tile_count[t] = 0;
  if (t < 4) F.scal[t] = 0;
}

__global__ void __launch_bounds__(kThreads) k_bin(FrameDev F) {
  bin_body(F, (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

__global__ void __launch_bounds__(kScanThreads) k_tile_scan(FrameDev F) {
  __shared__ long long buf[kScanChunk];
  __shared__ long long part[kScanThreads];
  tile_scan_body(F, buf, part);
}

// Inspection only: writes every tile's ids in ascending order at
// out_pids[tile_first .. + count) with their keys (when all pairs fit in
// `capacity`), and tile_start[0..n_tiles].  One wave per tile, the raster's sort;
// a tile whose bucket overflowed is rebuilt by scanning all particles in id
// order (ballot-compacted), as the raster visits them.
__global__ void __launch_bounds__(64) k_sort_segments(FrameDev F, int* __restrict__ out_keys,
                                                      int* __restrict__ out_pids, int64_t capacity,
                                                      int* __restrict__ tile_start) {
  __shared__ int seg[kSegSort];
  const int tile = blockIdx.x, lane = threadIdx.x;
  const int start = F.tile_first[tile];
  if (tile == 0 && lane == 0) tile_start[F.n_tiles] = F.scal[3];
  if (lane == 0) tile_start[tile] = start;
  if ((int64_t)F.scal[3] > capacity) return;  // the lists would not fit: left untouched
  const int cnt = F.tile_count[tile];
  const int cap = (int)F.cap;
  const int* __restrict__ bucket = F.pids + (int64_t)tile * cap;
  if (cnt <= cap && cnt <= 64) {
    const int v = wave_sort64(lane < cnt ? bucket[lane] : INT_MAX, lane);
    if (lane < cnt) out_pids[start + lane] = v;
  } else if (cnt <= cap) {
    int n2 = 128;
    while (n2 < cnt) n2 <<= 1;
    for (int i = lane; i < n2; i += 64) seg[i] = i < cnt ? bucket[i] : INT_MAX;
    __syncthreads();
    lds_sort(seg, n2, lane);
    for (int i = lane; i < cnt; i += 64) out_pids[start + i] = seg[i];
  } else {
    const int ty = tile / F.ntx, tx = tile - ty * F.ntx;
    const int x0 = tx * F.tile_w, x1 = x0 + F.tile_w - 1, y0 = ty * F.tile_h, y1 = y0 + F.tile_h - 1;
    const unsigned long long lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    int base = start;
    for (int64_t p0 = 0; p0 < F.n; p0 += 64) {
      const int64_t p = p0 + lane;
      bool hit = false;
      if (p < F.n) {
        const int4 b = F.boxes[p];
        hit = !(b.x > b.y || b.x > x1 || b.y < x0 || b.z > y1 || b.w < y0);
      }
      const unsigned long long m = __ballot(hit);
      if (hit) out_pids[base + __popcll(m & lt)] = (int)p;
      base += __popcll(m);
    }
  }
  for (int i = lane; i < cnt; i += 64) out_keys[start + i] = tile;
}

hipError_t launch_binning(const FramePlan& p, const float* soa, FrameBufs& b, hipStream_t s) {
  FrameDev F = make_dev(p, b);
  F.soa = soa;
  const unsigned gt = (unsigned)((p.n_tiles + kThreads - 1) / kThreads);
  const int64_t lanes = p.n * kBinGroup;
  const unsigned gp = (unsigned)(lanes > 0 ? (lanes + kThreads - 1) / kThreads : 1);
  hipLaunchKernelGGL(k_bin_clear, dim3(gt), dim3(kThreads), 0, s, F);
  hipLaunchKernelGGL(k_bin, dim3(gp), dim3(kThreads), 0, s, F);
  return hipGetLastError();
}

hipError_t launch_bin_outputs(const FramePlan& p, FrameBufs& b, int* keys_out, int* pids_out, int64_t capacity,
                              int* tile_start, hipStream_t s) {
  FrameDev F = make_dev(p, b);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kScanThreads), 0, s, F);
  hipLaunchKernelGGL(k_sort_segments, dim3(p.n_tiles), dim3(64), 0, s, F, keys_out, pids_out, capacity,
                     tile_start);
  return hipGetLastError();
}

}  // namespace osog
