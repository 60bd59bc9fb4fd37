// Integer tile binning of the particle table (steps F1-F4): a counting sort of
// the (tile key, particle id) pairs on the tile key, with exact segment offsets.
// The paper composes particle patches with an atomic scatter-add (Sec. III.C,
// Eq. 7); grouping the pairs by tile instead lets every tile sum its particles in
// LDS, in fixed point, with no global float atomics, so the canvas is bitwise
// reproducible.
//
//   k_bin_clear  tile histogram, slice counters and flags = 0
//   k_bin        F1: records, boxes, pairs per particle; tile histogram
//   k_tile_scan  F2: exclusive prefix of the histogram = each tile's segment start
//                (and the emit cursors); total pairs
//   k_emit       F3: every pair takes the next entry of its tile's segment
// The raster's fixed-point sums do not depend on the order inside a segment;
// k_sort_segments restores ascending id for the inspection API (F4).
// Integer atomics only form order-independent results (counts) or entries
// inside a tile's segment.  The pair list holds pair_cap entries: a tile whose
// segment does not fit is read by an id-ordered scan of all particles' boxes.
#include <hip/hip_runtime.h>

#include "osog_internal.h"
#include "stages.h"

namespace osog {

__global__ void __launch_bounds__(kThreads) k_bin_clear(FrameDev F) {
  const int t = blockIdx.x * kThreads + threadIdx.x;
  if (t < F.n_tiles) {
    F.tile_count[t] = 0;
    F.tile_done[t] = 0;
  }
  if (t < 4) F.scal[t] = 0;
}

__global__ void __launch_bounds__(kThreads) k_bin(FrameDev F) {
  bin_body(F, (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

__global__ void __launch_bounds__(kScanThreads) k_tile_scan(FrameDev F) {
  __shared__ long long wsum[2 * (kScanThreads / 64) + 1];
  tile_scan_body(F, wsum);
}

__global__ void __launch_bounds__(kThreads) k_emit(FrameDev F) {
  emit_body(F, (int64_t)blockIdx.x * kThreads + threadIdx.x);
}

// Inspection only: every tile's ids in ascending order at out_pids[tile_start ..
// + count) with their keys (when all pairs fit in `capacity`), and tile_start.
// One wave per tile, read exactly as the raster reads its segment.
__global__ void __launch_bounds__(64) k_sort_segments(FrameDev F, int* __restrict__ out_keys,
                                                      int* __restrict__ out_pids, int64_t capacity,
                                                      int* __restrict__ tile_start) {
  __shared__ int seg[kSegSort];  // 4 KB
  const int tile = blockIdx.x, lane = threadIdx.x;
  const int start = F.tile_start[tile];
  if (tile == 0 && lane == 0) tile_start[F.n_tiles] = F.tile_start[F.n_tiles];
  if (lane == 0) tile_start[tile] = start;
  if ((int64_t)F.tile_start[F.n_tiles] > capacity) return;  // the lists would not fit: left untouched
  int base = start;
  const TileIds T = tile_ids(F, tile, lane, seg, kSegSort);
  visit_tile_ids(F, tile, lane, T, [&](int mine, int m) {
    if (lane < m) {
      out_pids[base + lane] = mine;
      out_keys[base + lane] = tile;
    }
    base += m;
  });
}

hipError_t launch_binning(const FramePlan& p, const float* soa, FrameBufs& b, hipStream_t s) {
  FrameDev F = make_dev(p, b);
  F.soa = soa;
  const unsigned gt = (unsigned)((p.n_tiles + kThreads - 1) / kThreads);
  const int64_t lanes = p.n * kBinGroup;
  const unsigned ge = (unsigned)(lanes > 0 ? (lanes + kThreads - 1) / kThreads : 1);
  hipLaunchKernelGGL(k_bin_clear, dim3(gt), dim3(kThreads), 0, s, F);
  hipLaunchKernelGGL(k_bin, dim3(ge), dim3(kThreads), 0, s, F);
  hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kScanThreads), 0, s, F);
  hipLaunchKernelGGL(k_emit, dim3(ge), dim3(kThreads), 0, s, F);
  return hipGetLastError();
}

hipError_t launch_bin_outputs(const FramePlan& p, FrameBufs& b, int* keys_out, int* pids_out, int64_t capacity,
                              int* tile_start, hipStream_t s) {
  FrameDev F = make_dev(p, b);
  hipLaunchKernelGGL(k_sort_segments, dim3(p.n_tiles), dim3(64), 0, s, F, keys_out, pids_out, capacity,
                     tile_start);
  return hipGetLastError();
}

}  // namespace osog
