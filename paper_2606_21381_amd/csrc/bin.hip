// Integer tile binning of the particle table (steps F1-F4): per-particle pixel
// box -> pair counts -> particle-major emission of (tile key, particle id)
// pairs -> stable two-pass LSD radix sort on the tile key -> per-tile first and
// one-past-last sorted index.  The paper composes particle patches with an
// atomic scatter-add (Sec. III.C, Eq. 7); sorting the pairs instead lets every
// tile sum its particles in ascending id with no float atomics, so the canvas
// is bitwise reproducible.
//
// Six small kernels, none of them a single-workgroup scan (bodies in stages.h):
//   k_prepare   records, boxes, counts, per-block count sums; clears the
//               counters the later kernels accumulate into
//   k_emit      each block sums the preceding blocks' totals (its emission
//               offset), scans its own counts, emits its pairs and counts their
//               low key digit per 256-pair slice
//   k_digit_offsets + k_scatter (pass 0): stable scatter on the low digit;
//               counts the high digit per output slice
//   k_digit_offsets + k_scatter (pass 1): stable scatter on the high digit;
//               marks each tile's first and one-past-last sorted index
// Integer atomics only ever form order-independent results (sums, min, max).
#include <hip/hip_runtime.h>

#include "osog_internal.h"
#include "stages.h"

namespace osog {

__global__ void __launch_bounds__(kThreads) k_prepare(FrameDev F) {
  __shared__ __align__(16) char lds[2 * kThreads * sizeof(long long)];
  prepare_body(F, blockIdx.x, gridDim.x, lds);
}

__global__ void __launch_bounds__(kThreads) k_emit(FrameDev F) {
  __shared__ __align__(16) char lds[2 * kThreads * sizeof(long long)];
  emit_body(F, blockIdx.x, lds);
}

__global__ void __launch_bounds__(kThreads) k_digit_offsets(FrameDev F, int pass) {
  __shared__ __align__(16) char lds[kThreads * sizeof(int)];
  digit_offsets_body(F, pass, blockIdx.x, lds);
}

__global__ void __launch_bounds__(kThreads) k_scatter(FrameDev F, int pass) {
  __shared__ __align__(16) char lds[5 * 256 * sizeof(int)];
  scatter_body(F, pass, blockIdx.x, lds);
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
  FrameDev F = make_dev(p, b);
  F.soa = soa;
  const int gridp = F.nblk > 0 ? F.nblk : 1;
  hipLaunchKernelGGL(k_prepare, dim3(gridp), dim3(kThreads), 0, s, F);
  hipLaunchKernelGGL(k_emit, dim3(gridp), dim3(kThreads), 0, s, F);
  if (F.d1 > 0 && F.nblk > 0) {
    hipLaunchKernelGGL(k_digit_offsets, dim3(1 << F.d1), dim3(kThreads), 0, s, F, 0);
    hipLaunchKernelGGL(k_scatter, dim3(F.nsl), dim3(kThreads), 0, s, F, 0);
    if (F.d2 > 0) {
      hipLaunchKernelGGL(k_digit_offsets, dim3(1 << F.d2), dim3(kThreads), 0, s, F, 1);
      hipLaunchKernelGGL(k_scatter, dim3(F.nsl), dim3(kThreads), 0, s, F, 1);
    }
  }
  b.sorted_vals = F.sorted_vals;
  b.sorted_keys = (F.d1 > 0 && F.d2 == 0) ? b.keys_b : b.keys_a;
  return hipGetLastError();
}

hipError_t launch_tile_start(const FramePlan& p, FrameBufs& b, int* tile_start, hipStream_t s) {
  hipLaunchKernelGGL(k_tile_start, dim3((p.n_tiles + 1 + kThreads - 1) / kThreads), dim3(kThreads), 0,
                     s, b.sorted_keys, b.scal, p.n_tiles, tile_start);
  return hipGetLastError();
}

}  // namespace osog
