// OPD rasterisation (step F5): one 64-lane wave per tile, four pixels per lane.
// Absorbing frames also build the absorbance canvas tau = sum of dmu * thickness
// from the same coverage values, in the same order (the Beer-Lambert exponent of
// Eq. 4).
// Every pixel adds dn * thickness of each of its tile's particles in ascending
// particle id (the wave sorts its tile's ids first), so the sum order -- and the
// canvas, bit for bit -- does not depend on the tiling, the launch order or the GPU.  This replaces the
// paper's atomic scatter-add (Sec. III.C, Eq. 7) by a gather over the sorted
// pair list.  The particle id and its 128-byte record are wave-uniform and are
// read through the scalar cache; each 64-pixel slot first tests the particle
// against its own pixel rectangle (skip / full coverage), and both shortcuts
// return exactly what the per-pixel code would.  Body: raster_tile (stages.h).
#include <hip/hip_runtime.h>

#include "osog_internal.h"
#include "stages.h"

namespace osog {

// Workgroups are dealt to the 8 XCDs in turn (workgroup i to XCD i mod 8), so
// the tile of workgroup i is chosen to give each XCD one contiguous band of
// tiles: a particle spanning neighbouring tiles is then fetched into one L2.
// HAB: the frame's context defines polyhedral habits (a separate build of the
// kernel, so frames without them keep the smaller register footprint).
template <bool ABS, bool HAB>
__global__ void __launch_bounds__(64) k_raster(FrameDev F, int per_xcd) {
  __shared__ int seg[kSegSort];
  const int tile = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (tile < F.n_tiles) raster_tile<ABS, HAB>(F, tile, threadIdx.x, seg);
}

hipError_t launch_raster(const FramePlan& p, FrameBufs& b, float* opd, float* tau, hipStream_t s) {
  FrameDev F = make_dev(p, b);
  F.opd = opd;
  F.tau = tau;
  const int per = (p.n_tiles + kXcds - 1) / kXcds;
  const dim3 g(per * kXcds), wg(64);
  if (p.n_habits > 0) {
    if (p.absorb) hipLaunchKernelGGL((k_raster<true, true>), g, wg, 0, s, F, per);
    else hipLaunchKernelGGL((k_raster<false, true>), g, wg, 0, s, F, per);
  } else {
    if (p.absorb) hipLaunchKernelGGL((k_raster<true, false>), g, wg, 0, s, F, per);
    else hipLaunchKernelGGL((k_raster<false, false>), g, wg, 0, s, F, per);
  }
  return hipGetLastError();
}

}  // namespace osog
