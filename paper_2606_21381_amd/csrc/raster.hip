// OPD rasterisation (step F5): one workgroup per tile, one thread per pixel.
// The tile's particles, already sorted by id, are staged in LDS in chunks of
// 256 records; every pixel adds dn * thickness of each in ascending id, so the
// sum order -- and the canvas, bit for bit -- does not depend on the tiling,
// the launch order or the GPU.  This replaces the paper's atomic scatter-add
// (Sec. III.C, Eq. 7) by a gather over a sorted pair list.
#include <hip/hip_runtime.h>

#include "geometry.h"
#include "osog_internal.h"

namespace osog {

__global__ void __launch_bounds__(kThreads) k_raster(const int* __restrict__ tile_start,
                                                     const int* __restrict__ pids,
                                                     const PRec* __restrict__ recs,
                                                     const int4* __restrict__ boxes, int64_t n,
                                                     const int* __restrict__ scal, int W,
                                                     int tile_h, int tile_w, int ntx,
                                                     float* __restrict__ opd) {
  __shared__ PRec srec[kThreads];
  const int t = threadIdx.x, tile = blockIdx.x;
  const int ty = tile / ntx, tx = tile - ty * ntx;
  const int li = t / tile_w, lj = t - li * tile_w;
  const int i = ty * tile_h + li, j = tx * tile_w + lj;
  float acc = 0.0f;
  if (!scal[1]) {
    const int start = tile_start[tile], end = tile_start[tile + 1];
    for (int base = start; base < end; base += kThreads) {
      const int cnt = min(kThreads, end - base);
      if (t < cnt) srec[t] = recs[pids[base + t]];
      __syncthreads();
      for (int k = 0; k < cnt; ++k) acc += particle_opd(srec[k], i, j);
      __syncthreads();
    }
  } else {
    // Pair list overflowed its capacity: scan every particle in id order and
    // keep those whose box meets this tile (same boxes, same order, same sums).
    const int x0 = tx * tile_w, x1 = x0 + tile_w - 1, y0 = ty * tile_h, y1 = y0 + tile_h - 1;
    __shared__ int sel[kThreads];
    __shared__ int nsel;
    for (int64_t base = 0; base < n; base += kThreads) {
      if (t == 0) nsel = 0;
      __syncthreads();
      // ordered compaction: ballot within each wave, waves in order
      const int64_t p = base + t;
      bool hit = false;
      if (p < n) {
        int4 b = boxes[p];
        hit = b.x <= b.y && b.x <= x1 && b.y >= x0 && b.z <= y1 && b.w >= y0;
      }
      __shared__ int wc[kThreads / 64];
      const unsigned long long m = __ballot(hit);
      const int lane = t & 63, wave = t >> 6;
      if (lane == 0) wc[wave] = __popcll(m);
      __syncthreads();
      int off = 0;
      for (int w = 0; w < wave; ++w) off += wc[w];
      const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
      if (hit) sel[off + __popcll(m & lt)] = (int)p;
      if (t == 0) { int s = 0; for (int w = 0; w < kThreads / 64; ++w) s += wc[w]; nsel = s; }
      __syncthreads();
      const int cnt = nsel;
      if (t < cnt) srec[t] = recs[sel[t]];
      __syncthreads();
      for (int k = 0; k < cnt; ++k) acc += particle_opd(srec[k], i, j);
      __syncthreads();
    }
  }
  opd[(int64_t)i * W + j] = acc;
}

hipError_t launch_raster(const FramePlan& p, FrameBufs& b, float* opd, hipStream_t s) {
  hipLaunchKernelGGL(k_raster, dim3(p.n_tiles), dim3(kThreads), 0, s, b.tile_start, b.vals_a,
                     b.recs, b.boxes, p.n, b.scal, p.W, p.tile_h, p.tile_w, p.ntx, opd);
  return hipGetLastError();
}

}  // namespace osog
