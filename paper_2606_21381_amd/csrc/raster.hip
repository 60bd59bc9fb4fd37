// OPD rasterisation (step F5): one workgroup per tile, one thread per pixel.
// Every pixel adds dn * thickness of each of its tile's particles in ascending
// particle id, so the sum order -- and the canvas, bit for bit -- does not
// depend on the tiling, the launch order or the GPU.  This replaces the
// paper's atomic scatter-add (Sec. III.C, Eq. 7) by a gather over the sorted
// pair list.
//
// The particle id and its 64-byte record are wave-uniform, so they are read
// through the scalar cache (readfirstlane makes the address provably uniform);
// no LDS staging and no barriers.  Each wave first tests the particle against
// its own pixel rectangle: it skips particles whose per-pixel result would be
// exactly 0 everywhere, and adds amp directly where every pixel would be
// exactly fully covered -- both shortcuts return what the per-pixel code would.
#include <hip/hip_runtime.h>

#include "geometry.h"
#include "osog_internal.h"

namespace osog {

struct WaveRect {
  float x0, x1, y0, y1;  // pixel-edge bounds of the wave's pixels
};

__device__ __forceinline__ WaveRect wave_rect(int t, int tile_w, int tile_h, int tx, int ty) {
  const int w0 = t & ~63, w1 = w0 + 63;
  int r0 = w0 / tile_w, r1 = w1 / tile_w, c0 = 0, c1 = tile_w - 1;
  if (tile_w > 64) { c0 = w0 % tile_w; c1 = w1 % tile_w; }
  WaveRect R;
  R.x0 = (float)(tx * tile_w + c0);
  R.x1 = (float)(tx * tile_w + c1 + 1);
  R.y0 = (float)(ty * tile_h + r0);
  R.y1 = (float)(ty * tile_h + r1 + 1);
  return R;
}

// Contribution of one particle to this thread's pixel, with the wave-level shortcuts.
__device__ __forceinline__ float contribution(const PRec& r, const WaveRect& R, int i, int j) {
  const float kind = r.f[3];
  if (kind == 0.0f) {
    const float4 bb = prism_bounds(r);
    if (bb.y <= R.x0 || bb.x >= R.x1 || bb.w <= R.y0 || bb.z >= R.y1) return 0.0f;
    // all four corner pixel centres deep inside both slabs: every pixel has coverage 1
    const float m = 1e-4f;
    if (prism_classify(r, R.x0 + 0.5f, R.y0 + 0.5f, m) > 0 && prism_classify(r, R.x1 - 0.5f, R.y0 + 0.5f, m) > 0 &&
        prism_classify(r, R.x0 + 0.5f, R.y1 - 0.5f, m) > 0 && prism_classify(r, R.x1 - 0.5f, R.y1 - 0.5f, m) > 0)
      return r.f[2];
    return r.f[2] * prism_cover(r, bb, i, j);
  }
  if (kind == 1.0f) {
    const float2 ex = ellipse_extent(r);
    if (R.x1 - 0.5f - r.f[0] < -ex.x || R.x0 + 0.5f - r.f[0] > ex.x || R.y1 - 0.5f - r.f[1] < -ex.y ||
        R.y0 + 0.5f - r.f[1] > ex.y)
      return 0.0f;
    return ellipsoid_opd(r, i, j);
  }
  return 0.0f;
}

__global__ void __launch_bounds__(kThreads) k_raster(const int* __restrict__ tile_first,
                                                     const int* __restrict__ tile_count,
                                                     const int* __restrict__ pids,
                                                     const PRec* __restrict__ recs,
                                                     const int4* __restrict__ boxes, int64_t n,
                                                     const int* __restrict__ scal, int W,
                                                     int tile_h, int tile_w, int ntx,
                                                     float* __restrict__ opd) {
  const int t = threadIdx.x, tile = blockIdx.x;
  const int ty = tile / ntx, tx = tile - ty * ntx;
  const int li = t / tile_w, lj = t - li * tile_w;
  const int i = ty * tile_h + li, j = tx * tile_w + lj;
  const WaveRect R = wave_rect(t, tile_w, tile_h, tx, ty);
  float acc = 0.0f;
  if (!scal[1]) {
    const int cnt = tile_count[tile];
    const int start = cnt > 0 ? tile_first[tile] : 0;
    const int lane = t & 63;
    // up to 64 ids per vector load; each id is then broadcast with readlane and
    // the next record's scalar load is issued before the current one is used
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      const int m = min(64, cnt - c0);
      const int mine = lane < m ? pids[start + c0 + lane] : 0;
      PRec nxt = recs[__builtin_amdgcn_readlane(mine, 0)];
      for (int k = 0; k < m; ++k) {
        const PRec cur = nxt;
        if (k + 1 < m) nxt = recs[__builtin_amdgcn_readlane(mine, k + 1)];
        acc += contribution(cur, R, i, j);
      }
    }
  } else {
    // The pair list overflowed its capacity: visit every particle in id order and
    // keep those whose pixel box meets this tile (same records, same order, same sums).
    const int x0 = tx * tile_w, x1 = x0 + tile_w - 1, y0 = ty * tile_h, y1 = y0 + tile_h - 1;
    for (int64_t p = 0; p < n; ++p) {
      const int4 b = boxes[p];
      if (b.x > b.y || b.x > x1 || b.y < x0 || b.z > y1 || b.w < y0) continue;
      const PRec r = recs[p];
      acc += contribution(r, R, i, j);
    }
  }
  opd[(int64_t)i * W + j] = acc;
}

hipError_t launch_raster(const FramePlan& p, FrameBufs& b, float* opd, hipStream_t s) {
  hipLaunchKernelGGL(k_raster, dim3(p.n_tiles), dim3(kThreads), 0, s, b.tile_first, b.tile_count,
                     b.sorted_vals, b.recs, b.boxes, p.n, b.scal, p.W, p.tile_h, p.tile_w, p.ntx, opd);
  return hipGetLastError();
}

}  // namespace osog
