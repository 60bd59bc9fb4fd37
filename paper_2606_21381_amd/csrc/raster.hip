// OPD rasterisation (step F5): one workgroup per tile, one thread per pixel.
// Every pixel adds dn * thickness of each of its tile's particles in ascending
// particle id, so the sum order -- and the canvas, bit for bit -- does not
// depend on the tiling, the launch order or the GPU.  This replaces the
// paper's atomic scatter-add (Sec. III.C, Eq. 7) by a gather over the sorted
// pair list.
//
// The particle id and its 128-byte record are wave-uniform, so they are read
// through the scalar cache (readlane makes the address provably uniform); no
// LDS staging and no barriers.  Each 64-pixel slot first tests the particle
// against its own pixel rectangle: it skips particles whose per-pixel result
// would be exactly 0 everywhere, and adds amp directly where every pixel would
// be exactly fully covered -- both shortcuts return what the per-pixel code would.
#include <hip/hip_runtime.h>

#include "geometry.h"
#include "osog_internal.h"

namespace osog {

struct SubRect {
  float x0, x1, y0, y1;  // pixel-edge bounds of the 64 pixels one lane slot covers
};

__device__ __forceinline__ SubRect slot_rect(int first, int tile_w, int tx, int ty, int tile_h) {
  const int w0 = first, w1 = first + 63;
  int r0 = w0 / tile_w, r1 = w1 / tile_w, c0 = 0, c1 = tile_w - 1;
  if (tile_w > 64) { c0 = w0 % tile_w; c1 = w1 % tile_w; }
  SubRect R;
  R.x0 = (float)(tx * tile_w + c0);
  R.x1 = (float)(tx * tile_w + c1 + 1);
  R.y0 = (float)(ty * tile_h + r0);
  R.y1 = (float)(ty * tile_h + r1 + 1);
  return R;
}

// Contribution of one particle to one pixel of a 64-pixel slot, with the
// slot-level shortcuts (both give exactly what the per-pixel code would).
__device__ __forceinline__ float contribution(const PRec& r, const SubRect& R, int i, int j) {
  const float kind = r.f[3];
  if (kind == 0.0f) {
    if (r.f[21] <= R.x0 || r.f[20] >= R.x1 || r.f[23] <= R.y0 || r.f[22] >= R.y1) return 0.0f;
    // every pixel centre of the slot deep inside both slabs: coverage 1 everywhere
    // (max |u| over the rectangle of centres = |u at its middle| + |c| hx + |s| hy)
    const float c = r.f[4], s = r.f[5];
    const float hx = 0.5f * (R.x1 - R.x0 - 1.0f), hy = 0.5f * (R.y1 - R.y0 - 1.0f);
    const float dx = 0.5f * (R.x0 + R.x1) - r.f[0], dy = 0.5f * (R.y0 + R.y1) - r.f[1];
    const float ux = fabsf(c * dx + s * dy) + fabsf(c) * hx + fabsf(s) * hy;
    const float vy = fabsf(-s * dx + c * dy) + fabsf(s) * hx + fabsf(c) * hy;
    const float lim = 0.70712f + 1e-4f;
    if (ux < r.f[6] - lim && vy < r.f[7] - lim) return r.f[2];
    return r.f[2] * prism_cover(r, make_float4(r.f[20], r.f[21], r.f[22], r.f[23]), i, j);
  }
  if (kind == 1.0f) {
    if (R.x1 - 0.5f - r.f[0] < -r.f[16] || R.x0 + 0.5f - r.f[0] > r.f[16] || R.y1 - 0.5f - r.f[1] < -r.f[17] ||
        R.y0 + 0.5f - r.f[1] > r.f[17])
      return 0.0f;
    return ellipsoid_opd(r, i, j);
  }
  return 0.0f;
}

// One 64-lane wave per tile; lane l owns pixels l, l+64, l+128, l+192 of the
// tile (four slots of 64 pixels).  The particle loop, the record load and the
// kind dispatch run once per (tile, particle).
__global__ void __launch_bounds__(64) k_raster(const int* __restrict__ tile_first,
                                               const int* __restrict__ tile_end,
                                               const int* __restrict__ pids,
                                               const PRec* __restrict__ recs,
                                               const int4* __restrict__ boxes, int64_t n,
                                               const int* __restrict__ scal, int W, int tile_h,
                                               int tile_w, int ntx, float* __restrict__ opd) {
  const int lane = threadIdx.x, tile = blockIdx.x;
  const int ty = tile / ntx, tx = tile - ty * ntx;
  int pi[4], pj[4];
  SubRect R[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = lane + 64 * k, li = q / tile_w, lj = q - li * tile_w;
    pi[k] = ty * tile_h + li;
    pj[k] = tx * tile_w + lj;
    R[k] = slot_rect(64 * k, tile_w, tx, ty, tile_h);
  }
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (!scal[1]) {
    const int start = tile_first[tile];
    const int cnt = max(0, tile_end[tile] - start);
    // up to 64 ids per vector load; each id is then broadcast with readlane and
    // the next record's scalar load is issued before the current one is used
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      const int m = min(64, cnt - c0);
      const int mine = lane < m ? pids[start + c0 + lane] : 0;
      PRec nxt = recs[__builtin_amdgcn_readlane(mine, 0)];
      for (int k = 0; k < m; ++k) {
        const PRec cur = nxt;
        if (k + 1 < m) nxt = recs[__builtin_amdgcn_readlane(mine, k + 1)];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += contribution(cur, R[q], pi[q], pj[q]);
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
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += contribution(r, R[q], pi[q], pj[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) opd[(int64_t)pi[q] * W + pj[q]] = acc[q];
}

hipError_t launch_raster(const FramePlan& p, FrameBufs& b, float* opd, hipStream_t s) {
  hipLaunchKernelGGL(k_raster, dim3(p.n_tiles), dim3(64), 0, s, b.tile_first, b.tile_end,
                     b.sorted_vals, b.recs, b.boxes, p.n, b.scal, p.W, p.tile_h, p.tile_w, p.ntx, opd);
  return hipGetLastError();
}

}  // namespace osog
