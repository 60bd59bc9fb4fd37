// OPD rasterisation (step F5): one 64-lane wave per tile, the tile's pixel sums
// in LDS.  Absorbing frames also build the absorbance canvas tau = sum of
// dmu * thickness from the same coverage values (the Beer-Lambert exponent of
// Eq. 4).
// Each particle of the tile's segment deals the candidate pixels of its record
// that lie in the tile to the lanes, 64 at a time; the costly pixels (two prism
// edges, ellipse rim, habit face) are queued and evaluated 64 at a time.  The
// sums are 64-bit fixed point, so their order does not matter: every pixel's
// value depends only on the pixel and the particles that reach it, and the canvas
// is bitwise the same under every tiling, launch order and GPU.
// This replaces the paper's atomic scatter-add (Sec. III.C, Eq. 7) by a gather
// over the tile-sorted pair list.  Body: raster_tile (stages.h).
#include <hip/hip_runtime.h>

#include "osog_internal.h"
#include "stages.h"

namespace osog {

// Workgroups are dealt to the 8 XCDs in turn (workgroup i to XCD i mod 8), so
// the tile of workgroup i is chosen to give each XCD one contiguous band of
// tiles: a particle spanning neighbouring tiles is then fetched into one L2.
// HAB: the frame's context defines polyhedral habits (a separate build of the
// kernel, so frames without them keep the smaller register footprint).
// The first kSliceGrid workgroups take, in turn, the slices after the first of
// crowded tiles (so that they start early; a frame without crowded tiles costs
// kSliceGrid empty workgroups), the rest slice 0 of every tile.
constexpr int kSliceGrid = 4096;  // a multiple of kXcds

template <bool ABS, bool HAB>
__global__ void __launch_bounds__(64) k_raster(FrameDev F, int per_xcd) {
  extern __shared__ char lds_raster[];
  const int g = (int)blockIdx.x;
  if (g < kSliceGrid) {
    const int ne = F.scal[2];
    for (int e = g; e < ne; e += kSliceGrid) {
      const int it = F.items[e];
      if ((it & 15) == 0) continue;  // slice 0: the tile's own workgroup
      raster_tile<ABS, HAB>(F, it >> 4, it & 15, threadIdx.x, lds_raster);
      __syncthreads();  // the next slice reuses the LDS
    }
    return;
  }
  const int h = g - kSliceGrid;  // kSliceGrid is a multiple of kXcds: h mod 8 is still the XCD
  const int tile = (h % kXcds) * per_xcd + h / kXcds;
  if (tile < F.n_tiles) raster_tile<ABS, HAB>(F, tile, 0, threadIdx.x, lds_raster);
}

hipError_t launch_raster(const FramePlan& p, FrameBufs& b, float* opd, float* tau, hipStream_t s) {
  FrameDev F = make_dev(p, b);
  F.opd = opd;
  F.tau = tau;
  const int per = (p.n_tiles + kXcds - 1) / kXcds;
  const dim3 g((unsigned)(kSliceGrid + per * kXcds)), wg(64);
  const int area = p.tile_h * p.tile_w;
  const size_t lds = (size_t)raster_lds_bytes(area, p.absorb != 0);
  if (p.n_habits > 0) {
    if (p.absorb) hipLaunchKernelGGL((k_raster<true, true>), g, wg, lds, s, F, per);
    else hipLaunchKernelGGL((k_raster<false, true>), g, wg, lds, s, F, per);
  } else {
    if (p.absorb) hipLaunchKernelGGL((k_raster<true, false>), g, wg, lds, s, F, per);
    else hipLaunchKernelGGL((k_raster<false, false>), g, wg, lds, s, F, per);
  }
  return hipGetLastError();
}

}  // namespace osog
