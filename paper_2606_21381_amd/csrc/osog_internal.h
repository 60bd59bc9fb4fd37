// Internal declarations of libosog: device data structures, workspace plan and
// the kernel launchers shared between translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "osog.h"

namespace osog {

constexpr int kThreads = 256;     // every kernel runs 256-thread workgroups (4 wave64)
constexpr int kTwN = 4096;        // twiddle table length (largest FFT)
constexpr int kDefaultPairsPerParticle = 32;
constexpr int kXcds = 8;          // MI355X: 8 accelerator dies, each with its own L2
constexpr int kMinTile = 256;     // pixels per tile: a power of two in [kMinTile, kMaxTile]
constexpr int kMaxTile = 1024;
constexpr int kMaxHabits = 64;    // polyhedral habits per context
constexpr int kMaxFaces = 32;     // faces per habit

// Per-particle raster record, 128 bytes, written once by the prepare kernel and
// read by the raster through the scalar cache.
//   f[0] cx  f[1] cy  f[2] amp = dn*h (FP32)  f[3] kind (0 prism, 1 ellipsoid, -1 none)
//   f[4] cos f[5] sin f[6] a   f[7] b
//   prism     f[8..15]  footprint corner offsets from the centre (x0,y0,...,x3,y3), CCW
//             f[16..19] edge slopes dy/dx of edges 0-1, 1-2, 2-3, 3-0
//             f[20..23] footprint bounds xmin, xmax, ymin, ymax in canvas pixels
//             f[24..27] half-plane filter constants (p+q)/2, (p-q)/2, 1/p, 1/(2pq)
//                       with p = max(|cos|,|sin|), q = min (1/(2pq) kept finite)
//             f[28..31] candidate pixels (int bits): columns [jlo, jhi], rows [ilo, ihi] whose
//                       pixel square meets the bounds (not clamped to the canvas)
//   ellipsoid f[8] 1/a f[9] 1/b f[10..11] cos as double f[12..13] sin as double
//             f[14] dn f[15] h     (the FP64 rim refinement uses these)
//             f[16], f[17] half extents of the bounding box, enlarged (see ellipse_extent)
//             f[28..31] candidate pixels (int bits): columns [jlo, jhi], rows [ilo, ihi] whose
//                       centre lies inside the enlarged box (every other centre has q >= 1.002)
//   habit     (kind 2) as the ellipsoid in f[8..15]; f[16] = f[17] = max(a, b) R
//             (enlarged) bounds the solid's distance from the centre; f[18] habit index;
//             f[28..31] candidate pixels as for the ellipsoid
struct __align__(16) PRec {
  float f[32];
};

// Static per-call description of a frame, computed on the host.
struct FramePlan {
  int H, W, logH, logW;
  int tile_h, tile_w, ntx, nty, n_tiles;
  int kx_lo, kx_n;       // in-band signed kx range [kx_lo, kx_lo + kx_n)
  // incoherent DIC: the pupil's columns and the OTF's (|kx| up to twice the pupil's)
  int pup_lo, pup_n, otf_lo, otf_n;
  int rb;                // rows per band block of the blocked spectrum layout
  int fft_radix;         // FFT plan: largest Stockham radix (8 or 4)
  int64_t n, ld;         // particles, leading dimension
  int64_t pair_cap;      // entries of the pair list (pairs beyond it are not stored)
  // optics in the precision the kernels use
  int mode;
  float phase_k;         // 2 pi / lambda  [rad/um]
  float inv_lambda;      // 1 / lambda  [turns/um]
  float inv_wdx, inv_hdx;// 1/(W dx), 1/(H dx)  [cycles/um per bin]
  float kn;              // n_medium / lambda [cycles/um]
  float tfx, tfy;        // oblique tilt [cycles/um] (0 unless oblique)
  float cos_psi, sin_psi;// DIC shear direction
  float dx_um;
  double na_over_lambda; // pupil radius, FP64 (the band predicate is FP64)
  double dx_d, tfx_d, tfy_d;
  float photons;
  float read_sigma;      // Gaussian read noise [photon counts]
  // polyhedral habits of the context (device tables, kMaxFaces faces per habit):
  //   enc[f]  (p, q, r, type): type +1 / -1 an upper / lower bound W <= / >= p U + q V + r,
  //           type 0 a vertical face, inside where p U + q V + r <= 0
  //   raw[f]  (n_x, n_y, n_z, d) as given;  info[k] (faces, radius, topography amplitude, cell)
  const float4* hab_enc;
  const float4* hab_raw;
  const float4* hab_info;
  int n_habits;
  uint32_t topo_lo, topo_hi;
  uint32_t seed_lo, seed_hi, frame;
  int absorb;            // 1: Beer-Lambert amplitude from the absorbance canvas
};

// Carved views into the caller's workspace for one frame.
struct FrameBufs {
  PRec* recs;
  int4* boxes;
  int* counts;            // pairs per particle
  int* scal;              // [1] tiles rasterised by the id-ordered scan, [2] planes in use, [3] total pairs
  int* tile_count;        // n_tiles: pairs per tile (histogram)
  int* tile_start;        // n_tiles + 1: exclusive prefix of the tile counts
  int* cursor;            // n_tiles: next free entry of each tile's segment (emit)
  int* items;             // plane_count: (tile << 4 | slice) of every plane in use
  int* tile_plane;        // n_tiles: first plane of a sliced tile
  int* tile_done;         // n_tiles: slices finished (cleared per frame)
  unsigned long long* planes;  // plane_count planes of 2 * tile area: slices' fixed-point tile sums
  int* pids;              // pair_cap: particle ids, grouped by tile (segments at tile_start)
  float* opd;             // H*W (used when the caller passes no opd_out)
  float* tau;             // H*W absorbance (absorbing frames without opd_out)
  float2* absr;           // n: (dmu * height, dmu) per particle (absorbing frames)
  float2* band;           // H * W complex (blocked layout, kx_n used)
  double* colsum;         // W
  // backward only
  float2* band2;          // H * W complex
  float* gopd;            // H*W
  float* gtau;            // H*W: dL/dtau (absorbing frames)
  double* colgrad;        // 3 * W
  float2* otf;            // H*W: incoherent DIC spectra (blocked band layout)
  double* psum;           // H: incoherent DIC per-row-group sums
};

size_t frame_workspace_bytes(int H, int W, int64_t n, int tile_h, int tile_w, int ppp, bool backward);
FrameBufs carve(void* ws, int H, int W, int64_t n, int tile_h, int tile_w, int ppp, bool backward,
                int64_t* pair_cap_out);
// entries of the pair list: ppp pairs per particle plus one per tile
int64_t pair_capacity(int64_t n, int n_tiles, int ppp);
// planes of tile sums for the slices of crowded tiles (tiles past them are not
// sliced): a sliced tile of c > 48 stored pairs takes ceil(c / 48) <= c / 24 planes,
// so pair_cap / 24 + 1 bounds them; at most kPlaneBytes of planes (2 * area
// 64-bit sums each)
constexpr int64_t kPlaneBytes = int64_t(32) << 20;
int plane_count(int64_t pair_cap, int area);

// launchers (return hipError_t of the last launch)
hipError_t launch_binning(const FramePlan& p, const float* soa, FrameBufs& b, hipStream_t s);
hipError_t launch_bin_outputs(const FramePlan& p, FrameBufs& b, int* keys_out, int* pids_out, int64_t capacity,
                              int* tile_start, hipStream_t s);
// OPD into opd and, for absorbing frames, the absorbance into tau
hipError_t launch_raster(const FramePlan& p, FrameBufs& b, float* opd, float* tau, hipStream_t s);
hipError_t launch_pass1(const FramePlan& p, const float* opd, const float* tau, FrameBufs& b, const float2* tw,
                        hipStream_t s);
// pass 2 of a frame; band_in (if not null) is another band holding this frame's
// columns inside its range [in_kx_lo, in_kx_lo + in_kx_n) (a shared pass 1)
hipError_t launch_pass2(const FramePlan& p, const float* globals, FrameBufs& b, const float2* tw, hipStream_t s,
                        const float2* band_in = nullptr, int in_kx_lo = 0, int in_kx_n = 0);
hipError_t launch_pass3(const FramePlan& p, FrameBufs& b, const float2* tw, float* intensity, hipStream_t s,
                        int colsum_n = -1);
// incoherent DIC after passes 1 and 2 (full band, shear factor): |D|^2, its
// spectrum times the OTF of |h_obj|^2 (built here from the pupil), the image
hipError_t launch_incoherent_tail(const FramePlan& p, const float* globals, FrameBufs& b, const float2* tw,
                                  float* intensity, hipStream_t s);
hipError_t launch_philox(const uint32_t* ctr, int64_t count, uint32_t k0, uint32_t k1, uint32_t* out, hipStream_t s);

// backward launchers
hipError_t launch_pass2_keep(const FramePlan& p, const float* globals, FrameBufs& b, const float2* tw, hipStream_t s);
hipError_t launch_adj_pass3(const FramePlan& p, FrameBufs& b, const float2* tw, const float* grad_i, hipStream_t s);
hipError_t launch_adj_pass2(const FramePlan& p, const float* globals, FrameBufs& b, const float2* tw, hipStream_t s);
hipError_t launch_adj_pass1(const FramePlan& p, const float* opd, const float* tau, const float* grad_opd, FrameBufs& b,
                            const float2* tw, hipStream_t s);
hipError_t launch_raster_adjoint(const FramePlan& p, const float* soa, FrameBufs& b, float* grad_soa, hipStream_t s);
hipError_t launch_global_grads(const FramePlan& p, FrameBufs& b, float* grad_globals, hipStream_t s);

void set_error(const std::string& msg);

// spectral loss of Eq. 8 (spectral.hip)
size_t spectral_workspace_bytes(int H, int W);
hipError_t spectral_run(int H, int W, const float* img, const float* target, float* target_out, float eps,
                        float* loss, float* grad, void* ws, const float2* tw, hipStream_t s);

// learned initializer (cnn.hip)
int64_t cnn_param_count();
size_t cnn_workspace_bytes(int B, int H, int W);
hipError_t cnn_forward(int B, int H, int W, const float* images, const float* params, float* pred, void* ws,
                       hipStream_t s);
hipError_t cnn_train_step(int B, int H, int W, const float* images, const float* targets, float* params,
                          float* m, float* v, int step, float lr, float* loss, float* grads_out, void* ws,
                          hipStream_t s);
hipError_t conv3x3(int mode, int B, int Hi, int Wi, int Ci, int Co, int stride, const uint16_t* x,
                   const uint16_t* y, const uint16_t* gy, const uint16_t* w, const float* bias, uint16_t* out_bf16,
                   float* out_f32, void* ws, hipStream_t s);
size_t conv3x3_workspace_bytes(int mode, int B, int Hi, int Wi, int Ci, int Co, int stride);

struct Profiler;
// host helpers shared by the entry points (api.cpp)
FramePlan make_plan(const osog_context* ctx, int H, int W, int64_t n, int64_t ld, const osog_optics& o,
                    int64_t pair_cap);
hipError_t forward_frame(const osog_context* ctx, const FramePlan& p, const float* soa,
                         const float* globals, FrameBufs& b, float* opd_out, float* intensity,
                         hipStream_t s, bool profile);

// Stage profiler owned by the context (HIP events around stage launches).
struct Profiler;
Profiler* profiler_create();
void profiler_destroy(Profiler* p);
// begin/end return without doing anything when profiling is off
void profile_begin(Profiler* p, int stage, hipStream_t s);
void profile_end(Profiler* p, int stage, hipStream_t s);
void profiler_set(Profiler* p, bool on);
hipError_t profiler_read(Profiler* p, double* ms, int64_t* launches);

}  // namespace osog

// ---------------------------------------------------------------------------
// Device helpers shared by several kernels.
// ---------------------------------------------------------------------------
namespace osog {

__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
#pragma clang fp contract(off)
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): 10 rounds of two 32x32->64
// multiplies with the Weyl-sequence key schedule.  Each multiply is written as
// one 64-bit product so that it issues as a single v_mad_u64_u32 rather than a
// v_mul_hi_u32 / v_mul_lo_u32 pair.
__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t p0 = (uint64_t)M0 * c.x, p1 = (uint64_t)M1 * c.z;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    // x ^ y ^ z as one three-input logic op (truth table 0x96)
    c = make_uint4(__builtin_amdgcn_bitop3_b32(hi1, c.y, k0, 0x96), lo1, __builtin_amdgcn_bitop3_b32(hi0, c.w, k1, 0x96),
                   lo0);
    k0 += W0;
    k1 += W1;
  }
  return c;
}

__device__ __forceinline__ float u01(uint32_t x) {
  return ((float)(x >> 9) + 0.5f) * (1.0f / 8388608.0f);  // exact: 23-bit grid, never 0 or 1
}

}  // namespace osog
