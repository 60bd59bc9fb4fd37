// Host side of libosog: context, argument checks, frame planning, workspace
// carving and the C entry points declared in osog.h.
// Built with -ffp-contract=off: the pupil band bounds below must round exactly
// like the device predicate and the FP64 reference statement of the pupil.
#include <hip/hip_runtime.h>

#include <climits>
#include <algorithm>
#include <array>
#include <map>
#include <optional>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "batch.h"
#include "fft_common.h"
#include "osog.h"
#include "osog_internal.h"

struct osog_context {
  int device = 0;
  float2* twiddle = nullptr;  // kTwN entries: (cos, sin)(2 pi m / kTwN)
  int tile_h = 32, tile_w = 16;
  std::map<std::pair<int, int>, std::pair<int, int>> size_tiling;  // per canvas size (autotuner)
  std::map<std::pair<int, int>, int> size_radix;                   // per canvas size (autotuner)
  int fft_radix = 8;
  int batch_group = 4;
  osog::BatchCache* batch = nullptr;
  osog::Profiler* prof = nullptr;
  // polyhedral habits (osog_set_habits): enc, raw [kMaxHabits][kMaxFaces], info [kMaxHabits]
  float4* hab = nullptr;
  int n_habits = 0;
  uint64_t topo_seed = 0;
  uint64_t habit_gen = 0;  // bumped by every osog_set_habits: part of a captured batch's signature
  // device address of this GPU's copy of `scratch` (osog_render_noalloc), or NULL with the
  // error hipGetSymbolAddress returned
  void* scratch = nullptr;
  hipError_t scratch_err = hipSuccess;
};

// Fixed device scratch of osog_render_noalloc, for callers that cannot allocate.
// Every GPU that loads the library holds its own copy until the process ends.  In
// host code the name is only a stand-in for the symbol: kernels receive the device
// address that hipGetSymbolAddress returns for the current device (taken once per
// context in osog_context_create), never the name itself.
constexpr size_t kScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace osog {

static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }

static osog_status fail(osog_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}

static osog_status hip_fail(hipError_t e, const char* where) {
  return fail(OSOG_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

static bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

// Raster tiles: power-of-two sides, kMinTile..kMaxTile pixels (the raster's LDS sums)
static bool tile_shape_ok(int th, int tw) {
  return pow2_in(th, 1, kMaxTile) && pow2_in(tw, 1, kMaxTile) && th * tw >= kMinTile && th * tw <= kMaxTile;
}

static int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

static size_t align_up(size_t v) { return (v + 255) & ~size_t(255); }

// ---- workspace ---------------------------------------------------------------
struct Carver {
  char* base;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    T* p = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align_up(off + count * sizeof(T));
    return p;
  }
};

// Entries of the pair list: ppp pairs per particle plus one per tile (the
// tile-aligned part of every particle's box), at least one.
int plane_count(int64_t pair_cap, int area) {
  const int64_t c = pair_cap / 24 + 1, cap = kPlaneBytes / (16 * (int64_t)area);
  return (int)(c < cap ? c : cap);
}

int64_t pair_capacity(int64_t n, int n_tiles, int ppp) {
  const int64_t c = n * (int64_t)ppp + n_tiles;
  return c < 1 ? 1 : (c > INT_MAX ? INT_MAX : c);
}


static FrameBufs carve_impl(Carver& c, int H, int W, int64_t n, int tile_h, int tile_w, int ppp,
                            bool backward, int64_t* pair_cap_out) {
  const int n_tiles = (H / tile_h) * (W / tile_w);
  const int64_t pcap = pair_capacity(n, n_tiles, ppp);
  const size_t hw = (size_t)H * W;
  FrameBufs b{};
  b.recs = c.take<PRec>(n > 0 ? n : 1);
  b.boxes = c.take<int4>(n > 0 ? n : 1);
  b.counts = c.take<int>(n > 0 ? n : 1);
  b.scal = c.take<int>(64);
  b.tile_count = c.take<int>(n_tiles);
  b.tile_start = c.take<int>(n_tiles + 1);
  b.cursor = c.take<int>(n_tiles);
  const int npl = plane_count(pcap, tile_h * tile_w);
  b.items = c.take<int>(npl);
  b.tile_plane = c.take<int>(n_tiles);
  b.tile_done = c.take<int>(n_tiles);
  b.planes = c.take<unsigned long long>((size_t)npl * 2 * tile_h * tile_w);
  b.pids = c.take<int>((size_t)pcap);
  b.opd = c.take<float>(hw);
  b.tau = c.take<float>(hw);
  b.absr = c.take<float2>(n > 0 ? n : 1);
  b.band = c.take<float2>(hw);
  b.colsum = c.take<double>(W);
  if (backward) {
    b.band2 = c.take<float2>(hw);
    b.gopd = c.take<float>(hw);
    b.gtau = c.take<float>(hw);
    b.colgrad = c.take<double>(3 * (size_t)W);
    b.otf = c.take<float2>(hw);
    b.psum = c.take<double>(H);
  }
  if (pair_cap_out) *pair_cap_out = pcap;
  return b;
}

size_t frame_workspace_bytes(int H, int W, int64_t n, int tile_h, int tile_w, int ppp, bool backward) {
  Carver c{nullptr};
  carve_impl(c, H, W, n, tile_h, tile_w, ppp, backward, nullptr);
  return c.off;
}

FrameBufs carve(void* ws, int H, int W, int64_t n, int tile_h, int tile_w, int ppp, bool backward,
                int64_t* pair_cap_out) {
  Carver c{static_cast<char*>(ws)};
  return carve_impl(c, H, W, n, tile_h, tile_w, ppp, backward, pair_cap_out);
}

// Forward-only buffers of one frame, packed for the fixed scratch: the band keeps
// only the in-band columns, the OPD and absorbance planes exist only when the
// caller passes no opd_out, and the inspection prefix is left out.
static FrameBufs carve_compact(Carver& c, const FramePlan& p, int64_t pair_cap, bool own_opd) {
  const size_t hw = (size_t)p.H * p.W, nn = p.n > 0 ? (size_t)p.n : 1;
  const size_t kx = p.kx_n > 0 ? (size_t)p.kx_n : 1;
  FrameBufs b{};
  b.recs = c.take<PRec>(nn);
  b.boxes = c.take<int4>(nn);
  b.counts = c.take<int>(nn);
  b.scal = c.take<int>(64);
  b.tile_count = c.take<int>(p.n_tiles);
  b.tile_start = c.take<int>(p.n_tiles + 1);
  b.cursor = c.take<int>(p.n_tiles);
  const int npl = plane_count(pair_cap, p.tile_h * p.tile_w);
  b.items = c.take<int>(npl);
  b.tile_plane = c.take<int>(p.n_tiles);
  b.tile_done = c.take<int>(p.n_tiles);
  b.planes = c.take<unsigned long long>((size_t)npl * (p.absorb ? 2 : 1) * p.tile_h * p.tile_w);
  b.pids = c.take<int>((size_t)pair_cap);
  if (own_opd) {
    b.opd = c.take<float>(hw);
    if (p.absorb) b.tau = c.take<float>(hw);
  }
  if (p.absorb) b.absr = c.take<float2>(nn);
  b.band = c.take<float2>((size_t)p.H * kx);
  b.colsum = c.take<double>(kx);
  return b;
}

// ---- pupil band: signed kx columns with any bin inside the (shifted) disc ----
static void pupil_range(int H, int W, const osog_optics& o, int* kx_lo, int* kx_n) {
  const double vx = 1.0 / ((double)W * o.pixel_um), vy = 1.0 / ((double)H * o.pixel_um);
  const double tx = o.mode == OSOG_OBLIQUE ? o.tilt_fx : 0.0;
  const double ty = o.mode == OSOG_OBLIQUE ? o.tilt_fy : 0.0;
  const double r = o.na / o.wavelength_um, r2 = r * r;
  const int kmin = -(H / 2), kmax = H / 2 - 1;
  const double cky = -ty / vy;
  int c0 = (int)std::floor(cky);
  c0 = c0 < kmin ? kmin : (c0 > kmax ? kmax : c0);
  int c1 = c0 + 1 > kmax ? kmax : c0 + 1;
  int lo = INT_MAX, hi = INT_MIN;
  for (int kx = -(W / 2); kx < W / 2; ++kx) {
    const double gx = (double)kx * vx + tx;
    const double gx2 = gx * gx;
    const double gy0 = (double)c0 * vy + ty, gy1 = (double)c1 * vy + ty;
    if (gx2 + gy0 * gy0 <= r2 || gx2 + gy1 * gy1 <= r2) {
      if (kx < lo) lo = kx;
      if (kx > hi) hi = kx;
    }
  }
  if (lo > hi) { *kx_lo = 0; *kx_n = 0; }
  else { *kx_lo = lo; *kx_n = hi - lo + 1; }
}

// Columns passes 1 and 2 carry: the pupil's, or every column for the incoherent
// DIC (its shear acts before the pupil, on the whole spectrum).
static void band_range(int H, int W, const osog_optics& o, int* kx_lo, int* kx_n) {
  if (o.mode == OSOG_DIC_INCOHERENT) {
    *kx_lo = -(W / 2);
    *kx_n = W;
    return;
  }
  pupil_range(H, W, o, kx_lo, kx_n);
}

// Incoherent DIC: the OTF is the pupil's autocorrelation, non-zero only for |kx|
// up to twice the pupil's largest |kx|.
static void otf_range(int W, int pup_lo, int pup_n, int* lo, int* n) {
  if (pup_n == 0) { *lo = 0; *n = 0; return; }
  const int kmax = std::max(-pup_lo, pup_lo + pup_n - 1);
  if (4 * kmax + 1 >= W) { *lo = -(W / 2); *n = W; return; }
  *lo = -2 * kmax;
  *n = 4 * kmax + 1;
}

static osog_status check_optics(const osog_optics* o) {
  if (!o) return fail(OSOG_ERR_INVALID_ARGUMENT, "optics is NULL");
  if (o->mode < OSOG_BRIGHTFIELD || o->mode > OSOG_DIC_INCOHERENT)
    return fail(OSOG_ERR_INVALID_ARGUMENT,
                "optics.mode must be 0 (brightfield), 1 (DIC), 2 (oblique) or 3 (incoherent DIC)");
  if (!(o->wavelength_um > 0.0) || !std::isfinite(o->wavelength_um))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "optics.wavelength_um must be finite and > 0");
  if (!(o->pixel_um > 0.0) || !std::isfinite(o->pixel_um))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "optics.pixel_um must be finite and > 0");
  if (!(o->n_medium > 0.0) || !std::isfinite(o->n_medium))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "optics.n_medium must be finite and > 0");
  if (!(o->na > 0.0) || !(o->na < o->n_medium))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "optics.na must satisfy 0 < na < n_medium");
  if (!std::isfinite(o->shear_angle_rad) || !std::isfinite(o->tilt_fx) || !std::isfinite(o->tilt_fy))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "optics shear angle and tilt must be finite");
  if (!(o->photons_mean >= 0.0) || !std::isfinite(o->photons_mean))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "optics.photons_mean must be finite and >= 0");
  if (!(o->read_noise >= 0.0) || !std::isfinite(o->read_noise))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "optics.read_noise must be finite and >= 0");
  if (o->read_noise > 0.0 && !(o->photons_mean > 0.0))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "optics.read_noise needs photons_mean > 0 (it is in photon counts)");
  if (o->absorption != 0 && o->absorption != 1)
    return fail(OSOG_ERR_INVALID_ARGUMENT, "optics.absorption must be 0 or 1");
  return OSOG_OK;
}

void context_tiling(const osog_context* ctx, int H, int W, int* th, int* tw);
int context_radix(const osog_context* ctx, int H, int W);

static osog_status check_frame(const osog_context* ctx, int H, int W, const float* soa, int64_t n,
                               int64_t ld, const osog_optics* optics, const float* globals) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (n < 0 || n > INT_MAX) return fail(OSOG_ERR_INVALID_ARGUMENT, "n must be in [0, 2^31)");
  if (ld < n) return fail(OSOG_ERR_INVALID_ARGUMENT, "ld must be >= n");
  if (n > 0 && !soa) return fail(OSOG_ERR_INVALID_ARGUMENT, "soa is NULL");
  if (!globals) return fail(OSOG_ERR_INVALID_ARGUMENT, "globals is NULL");
  osog_status st = check_optics(optics);
  if (st != OSOG_OK) return st;
  if (!pow2_in(H, 32, 4096) || !pow2_in(W, 32, 4096))
    return fail(OSOG_ERR_UNSUPPORTED, "height and width must be powers of two in [32, 4096]");
  int th, tw;
  context_tiling(ctx, H, W, &th, &tw);
  if (H % th || W % tw) return fail(OSOG_ERR_UNSUPPORTED, "canvas sides must be multiples of the tile sides");
  return OSOG_OK;
}

void context_tiling(const osog_context* ctx, int H, int W, int* th, int* tw) {
  auto it = ctx->size_tiling.find({H, W});
  if (it != ctx->size_tiling.end()) { *th = it->second.first; *tw = it->second.second; }
  else { *th = ctx->tile_h; *tw = ctx->tile_w; }
}
int context_radix(const osog_context* ctx, int H, int W) {
  auto it = ctx->size_radix.find({H, W});
  return it != ctx->size_radix.end() ? it->second : ctx->fft_radix;
}
const float2* context_twiddle(const osog_context* ctx) { return ctx->twiddle; }
int context_device(const osog_context* ctx) { return ctx->device; }
BatchCache* context_batch(osog_context* ctx) { return ctx->batch; }
uint64_t context_habit_generation(const osog_context* ctx) { return ctx->habit_gen; }

FramePlan make_plan(const osog_context* ctx, int H, int W, int64_t n, int64_t ld,
                    const osog_optics& o, int64_t pair_cap) {
  FramePlan p{};
  p.H = H; p.W = W; p.logH = ilog2(H); p.logW = ilog2(W);
  context_tiling(ctx, H, W, &p.tile_h, &p.tile_w);
  p.ntx = W / p.tile_w; p.nty = H / p.tile_h; p.n_tiles = p.ntx * p.nty;
  band_range(H, W, o, &p.kx_lo, &p.kx_n);
  if (o.mode == OSOG_DIC_INCOHERENT) {
    pupil_range(H, W, o, &p.pup_lo, &p.pup_n);
    otf_range(W, p.pup_lo, p.pup_n, &p.otf_lo, &p.otf_n);
  }
  p.rb = rows_per_block(W);
  p.fft_radix = context_radix(ctx, H, W);
  p.n = n; p.ld = ld; p.pair_cap = pair_cap;
  p.mode = o.mode;
  p.phase_k = (float)(2.0 * M_PI / o.wavelength_um);
  p.inv_lambda = (float)(1.0 / o.wavelength_um);
  p.inv_wdx = (float)(1.0 / ((double)W * o.pixel_um));
  p.inv_hdx = (float)(1.0 / ((double)H * o.pixel_um));
  p.kn = (float)(o.n_medium / o.wavelength_um);
  p.tfx_d = o.mode == OSOG_OBLIQUE ? o.tilt_fx : 0.0;
  p.tfy_d = o.mode == OSOG_OBLIQUE ? o.tilt_fy : 0.0;
  p.tfx = (float)p.tfx_d; p.tfy = (float)p.tfy_d;
  p.cos_psi = (float)std::cos(o.shear_angle_rad);
  p.sin_psi = (float)std::sin(o.shear_angle_rad);
  p.dx_um = (float)o.pixel_um;
  p.dx_d = o.pixel_um;
  p.na_over_lambda = o.na / o.wavelength_um;
  p.photons = (float)o.photons_mean;
  p.read_sigma = (float)o.read_noise;
  p.seed_lo = (uint32_t)(o.seed & 0xffffffffu);
  p.seed_hi = (uint32_t)(o.seed >> 32);
  p.frame = o.noise_frame;
  p.absorb = o.absorption ? 1 : 0;
  p.n_habits = ctx->n_habits;
  p.hab_enc = ctx->hab;
  p.hab_raw = ctx->hab ? ctx->hab + kMaxHabits * kMaxFaces : nullptr;
  p.hab_info = ctx->hab ? ctx->hab + 2 * kMaxHabits * kMaxFaces : nullptr;
  p.topo_lo = (uint32_t)(ctx->topo_seed & 0xffffffffu);
  p.topo_hi = (uint32_t)(ctx->topo_seed >> 32);
  return p;
}

static int tile_of(const osog_context* ctx, int H, int W, int which) {
  int th, tw;
  context_tiling(ctx, H, W, &th, &tw);
  return which == 0 ? th : tw;
}

static int effective_ppp(int ppp) { return ppp > 0 ? ppp : kDefaultPairsPerParticle; }

// Forward chain of one frame on a carved workspace.
hipError_t forward_frame(const osog_context* ctx, const FramePlan& p, const float* soa,
                         const float* globals, FrameBufs& b, float* opd_out, float* intensity,
                         hipStream_t s, bool profile) {
  float* opd = opd_out ? opd_out : b.opd;
  float* tau = opd_out ? opd_out + (size_t)p.H * p.W : b.tau;  // absorbing frames: second plane
  Profiler* pr = profile ? ctx->prof : nullptr;
  hipError_t e;
  profile_begin(pr, OSOG_STAGE_BINNING, s);
  if ((e = launch_binning(p, soa, b, s)) != hipSuccess) return e;
  profile_end(pr, OSOG_STAGE_BINNING, s);
  profile_begin(pr, OSOG_STAGE_RASTER, s);
  if ((e = launch_raster(p, b, opd, tau, s)) != hipSuccess) return e;
  profile_end(pr, OSOG_STAGE_RASTER, s);
  profile_begin(pr, OSOG_STAGE_PASS1, s);
  if ((e = launch_pass1(p, opd, tau, b, ctx->twiddle, s)) != hipSuccess) return e;
  profile_end(pr, OSOG_STAGE_PASS1, s);
  if (p.kx_n > 0) {
    profile_begin(pr, OSOG_STAGE_PASS2, s);
    if ((e = launch_pass2(p, globals, b, ctx->twiddle, s)) != hipSuccess) return e;
    profile_end(pr, OSOG_STAGE_PASS2, s);
  }
  profile_begin(pr, OSOG_STAGE_PASS3, s);
  if (p.mode == OSOG_DIC_INCOHERENT) e = launch_incoherent_tail(p, globals, b, ctx->twiddle, intensity, s);
  else e = launch_pass3(p, b, ctx->twiddle, intensity, s);
  if (e != hipSuccess) return e;
  profile_end(pr, OSOG_STAGE_PASS3, s);
  return hipSuccess;
}

}  // namespace osog

using namespace osog;

extern "C" {

osog_status osog_context_create(osog_context** out, int device) {
  if (!out) return fail(OSOG_ERR_INVALID_ARGUMENT, "out is NULL");
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
  if (device < 0 || device >= count) return fail(OSOG_ERR_INVALID_ARGUMENT, "no such HIP device");
  if ((e = hipSetDevice(device)) != hipSuccess) return hip_fail(e, "hipSetDevice");
  osog_context* ctx = new (std::nothrow) osog_context();
  if (!ctx) return fail(OSOG_ERR_INVALID_ARGUMENT, "out of host memory");
  ctx->device = device;
  std::vector<float2> tw(kTwN);
  for (int m = 0; m < kTwN; ++m) {
    double a = 2.0 * M_PI * (double)m / (double)kTwN;
    tw[m] = make_float2((float)std::cos(a), (float)std::sin(a));
  }
  if ((e = hipMalloc(&ctx->twiddle, sizeof(float2) * kTwN)) != hipSuccess) {
    delete ctx;
    return hip_fail(e, "hipMalloc(twiddle)");
  }
  if ((e = hipMemcpy(ctx->twiddle, tw.data(), sizeof(float2) * kTwN, hipMemcpyHostToDevice)) != hipSuccess) {
    (void)hipFree(ctx->twiddle);
    delete ctx;
    return hip_fail(e, "hipMemcpy(twiddle)");
  }
  // this device's copy of the no-allocation scratch (the device is current here)
  ctx->scratch_err = hipGetSymbolAddress(&ctx->scratch, HIP_SYMBOL(scratch));
  if (ctx->scratch_err != hipSuccess) {
    ctx->scratch = nullptr;
    (void)hipGetLastError();  // keep the failure out of later launch checks
  }
  ctx->batch = batch_cache_create();
  ctx->prof = profiler_create();
  *out = ctx;
  return OSOG_OK;
}

osog_status osog_context_destroy(osog_context* ctx) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  (void)hipSetDevice(ctx->device);
  batch_cache_destroy(ctx->batch);
  profiler_destroy(ctx->prof);
  if (ctx->twiddle) (void)hipFree(ctx->twiddle);
  if (ctx->hab) (void)hipFree(ctx->hab);
  delete ctx;
  return OSOG_OK;
}

// Vertices of {x : A x <= d} by intersecting every triple of face planes (FP64),
// inside a guard box |x_i| <= 1e4 whose own faces are added: a vertex on the guard
// box means the habit is unbounded.
static bool habit_vertices(const float* f, int m, double* max_r, bool* bounded) {
  std::vector<std::array<double, 4>> F;
  for (int k = 0; k < m; ++k) F.push_back({f[4 * k], f[4 * k + 1], f[4 * k + 2], f[4 * k + 3]});
  const double G = 1e4;
  for (int ax = 0; ax < 3; ++ax)
    for (int sg = -1; sg <= 1; sg += 2) {
      std::array<double, 4> g{0, 0, 0, G};
      g[ax] = sg;
      F.push_back(g);
    }
  const int M = (int)F.size();
  int found = 0;
  *max_r = 0.0;
  *bounded = true;
  for (int a = 0; a < M; ++a)
    for (int b = a + 1; b < M; ++b)
      for (int c = b + 1; c < M; ++c) {
        const double* A[3] = {F[a].data(), F[b].data(), F[c].data()};
        const double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) -
                           A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
                           A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
        if (std::fabs(det) < 1e-12) continue;
        double x[3];
        for (int col = 0; col < 3; ++col) {  // Cramer's rule
          double Bm[3][3];
          for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) Bm[r][q] = q == col ? A[r][3] : A[r][q];
          x[col] = (Bm[0][0] * (Bm[1][1] * Bm[2][2] - Bm[1][2] * Bm[2][1]) -
                    Bm[0][1] * (Bm[1][0] * Bm[2][2] - Bm[1][2] * Bm[2][0]) +
                    Bm[0][2] * (Bm[1][0] * Bm[2][1] - Bm[1][1] * Bm[2][0])) / det;
        }
        bool in = true;
        for (int k = 0; k < M && in; ++k)
          in = F[k][0] * x[0] + F[k][1] * x[1] + F[k][2] * x[2] <= F[k][3] + 1e-7 * (1.0 + std::fabs(F[k][3]));
        if (!in) continue;
        ++found;
        if (a >= m || b >= m || c >= m) *bounded = false;
        *max_r = std::max(*max_r, std::sqrt(x[0] * x[0] + x[1] * x[1]));
      }
  return found >= 4;
}

osog_status osog_set_tiling(osog_context* ctx, int32_t tile_h, int32_t tile_w) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (!tile_shape_ok(tile_h, tile_w))
    return fail(OSOG_ERR_UNSUPPORTED, "tile sides must be powers of two with 256 <= tile_h * tile_w <= 1024");
  ctx->tile_h = tile_h;
  ctx->tile_w = tile_w;
  return OSOG_OK;
}

osog_status osog_get_tiling(const osog_context* ctx, int32_t* tile_h, int32_t* tile_w) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (!tile_h || !tile_w) return fail(OSOG_ERR_INVALID_ARGUMENT, "output pointer is NULL");
  *tile_h = ctx->tile_h;
  *tile_w = ctx->tile_w;
  return OSOG_OK;
}

osog_status osog_workspace_size(const osog_context* ctx, int32_t height, int32_t width, int64_t n,
                                int32_t pairs_per_particle, int32_t with_backward, size_t* bytes) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (!bytes) return fail(OSOG_ERR_INVALID_ARGUMENT, "bytes is NULL");
  if (n < 0 || n > INT_MAX) return fail(OSOG_ERR_INVALID_ARGUMENT, "n must be in [0, 2^31)");
  if (pairs_per_particle < 0) return fail(OSOG_ERR_INVALID_ARGUMENT, "pairs_per_particle must be >= 0");
  if (!pow2_in(height, 32, 4096) || !pow2_in(width, 32, 4096))
    return fail(OSOG_ERR_UNSUPPORTED, "height and width must be powers of two in [32, 4096]");
  if (height % tile_of(ctx, height, width, 0) || width % tile_of(ctx, height, width, 1))
    return fail(OSOG_ERR_UNSUPPORTED, "canvas sides must be multiples of the tile sides");
  *bytes = frame_workspace_bytes(height, width, n, tile_of(ctx, height, width, 0), tile_of(ctx, height, width, 1),
                                 effective_ppp(pairs_per_particle), with_backward != 0);
  return OSOG_OK;
}

osog_status osog_render(osog_context* ctx, void* stream, int32_t height, int32_t width,
                        const float* soa, int64_t n, int64_t ld, const osog_optics* optics,
                        const float* globals, float* opd_out, float* intensity_out,
                        void* workspace, size_t workspace_bytes) {
  osog_status st = check_frame(ctx, height, width, soa, n, ld, optics, globals);
  if (st != OSOG_OK) return st;
  if (!intensity_out) return fail(OSOG_ERR_INVALID_ARGUMENT, "intensity_out is NULL");
  if (!workspace) return fail(OSOG_ERR_WORKSPACE, "workspace is NULL");
  const bool big = optics->mode == OSOG_DIC_INCOHERENT;  // needs the spectra buffers of the larger carve
  // the largest pair capacity this workspace holds
  int ppp = 0;
  for (int cand = 1 << 20; cand >= 1; cand >>= 1)
    if (frame_workspace_bytes(height, width, n, tile_of(ctx, height, width, 0), tile_of(ctx, height, width, 1), cand, big) <= workspace_bytes) {
      ppp = cand;
      break;
    }
  if (ppp == 0)
    return fail(OSOG_ERR_WORKSPACE, big ? "incoherent DIC needs osog_workspace_size(with_backward=1) bytes"
                                        : "workspace smaller than osog_workspace_size()");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  int64_t cap = 0;
  FrameBufs b = carve(workspace, height, width, n, tile_of(ctx, height, width, 0), tile_of(ctx, height, width, 1), ppp, big, &cap);
  FramePlan p = make_plan(ctx, height, width, n, ld, *optics, cap);
  e = forward_frame(ctx, p, soa, globals, b, opd_out, intensity_out, (hipStream_t)stream, true);
  if (e != hipSuccess) return hip_fail(e, "osog_render launch");
  return OSOG_OK;
}

osog_status osog_render_noalloc(osog_context* ctx, void* stream, int32_t height, int32_t width,
                                const float* soa, int64_t n, int64_t ld, const osog_optics* optics,
                                const float* globals, float* opd_out, float* intensity_out) {
  osog_status st = check_frame(ctx, height, width, soa, n, ld, optics, globals);
  if (st != OSOG_OK) return st;
  if (!intensity_out) return fail(OSOG_ERR_INVALID_ARGUMENT, "intensity_out is NULL");
  if (optics->mode == OSOG_DIC_INCOHERENT)
    return fail(OSOG_ERR_UNSUPPORTED, "osog_render_noalloc does not render the incoherent DIC "
                                      "(its full spectra need osog_render's workspace)");
  if (!ctx->scratch)
    return fail(OSOG_ERR_HIP, std::string("no device address for the scratch: ") + hipGetErrorString(ctx->scratch_err));
  FramePlan p = make_plan(ctx, height, width, n, ld, *optics, 0);
  const bool own_opd = opd_out == nullptr;
  // the largest pair list that fits (results do not depend on it), up to 1024 pairs per particle
  int64_t cap = 0;
  size_t need = 0;
  for (int cand = 1024; cand >= 1; cand >>= 1) {
    const int64_t c = pair_capacity(n, p.n_tiles, cand);
    Carver probe{nullptr};
    carve_compact(probe, p, c, own_opd);
    need = probe.off;
    if (need <= kScratchBytes) {
      cap = c;
      break;
    }
  }
  if (cap == 0)
    return fail(OSOG_ERR_WORKSPACE, "frame needs " + std::to_string(need) + " bytes of scratch; osog_render_noalloc holds " +
                                        std::to_string(kScratchBytes) + " (use osog_render with a workspace)");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  Carver c{static_cast<char*>(ctx->scratch)};
  FrameBufs b = carve_compact(c, p, cap, own_opd);
  p.pair_cap = cap;
  e = forward_frame(ctx, p, soa, globals, b, opd_out, intensity_out, (hipStream_t)stream, false);
  if (e != hipSuccess) return hip_fail(e, "osog_render_noalloc launch");
  return OSOG_OK;
}

osog_status osog_render_multi(osog_context* ctx, void* stream, int32_t height, int32_t width,
                              const float* soa, int64_t n, int64_t ld, int32_t n_modes,
                              const osog_optics* optics, const float* globals, float* const* intensity_out,
                              float* opd_out, void* workspace, size_t workspace_bytes) {
  if (n_modes < 1 || n_modes > 64 || !optics || !intensity_out)
    return fail(OSOG_ERR_INVALID_ARGUMENT, "need 1 <= n_modes <= 64, optics[n_modes] and intensity_out[n_modes]");
  if (!globals) return fail(OSOG_ERR_INVALID_ARGUMENT, "globals is NULL");
  for (int m = 0; m < n_modes; ++m) {
    osog_status st = check_frame(ctx, height, width, soa, n, ld, &optics[m], globals + 4 * m);
    if (st != OSOG_OK) return fail(st, "mode " + std::to_string(m) + ": " + g_last_error);
    if (optics[m].mode == OSOG_DIC_INCOHERENT)
      return fail(OSOG_ERR_UNSUPPORTED, "osog_render_multi: the incoherent DIC renders through osog_render");
    if (!intensity_out[m]) return fail(OSOG_ERR_INVALID_ARGUMENT, "intensity_out[" + std::to_string(m) + "] is NULL");
    if (optics[m].wavelength_um != optics[0].wavelength_um || optics[m].pixel_um != optics[0].pixel_um ||
        optics[m].n_medium != optics[0].n_medium || optics[m].absorption != optics[0].absorption)
      return fail(OSOG_ERR_INVALID_ARGUMENT,
                  "all modes must share wavelength_um, pixel_um, n_medium and absorption");
  }
  if (!workspace) return fail(OSOG_ERR_WORKSPACE, "workspace is NULL");
  const int th = tile_of(ctx, height, width, 0), tw = tile_of(ctx, height, width, 1);
  int ppp = 0;
  for (int cand = 1 << 20; cand >= 1; cand >>= 1)
    if (frame_workspace_bytes(height, width, n, th, tw, cand, true) <= workspace_bytes) {
      ppp = cand;
      break;
    }
  if (ppp == 0) return fail(OSOG_ERR_WORKSPACE, "workspace smaller than osog_workspace_size(with_backward=1)");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  int64_t cap = 0;
  FrameBufs b = carve(workspace, height, width, n, th, tw, ppp, true, &cap);
  std::vector<FramePlan> plans;
  int lo = INT_MAX, hi = INT_MIN;
  for (int m = 0; m < n_modes; ++m) {
    plans.push_back(make_plan(ctx, height, width, n, ld, optics[m], cap));
    if (plans.back().kx_n > 0) {
      lo = std::min(lo, plans.back().kx_lo);
      hi = std::max(hi, plans.back().kx_lo + plans.back().kx_n - 1);
    }
  }
  // pass 1 once, over the union of the modes' in-band columns
  FramePlan u = plans[0];
  u.kx_lo = lo <= hi ? lo : 0;
  u.kx_n = lo <= hi ? hi - lo + 1 : 0;
  hipStream_t s = (hipStream_t)stream;
  float* opd = opd_out ? opd_out : b.opd;
  float* tau = opd_out ? opd_out + (size_t)height * width : b.tau;
  if ((e = launch_binning(u, soa, b, s)) != hipSuccess) return hip_fail(e, "osog_render_multi: binning");
  if ((e = launch_raster(u, b, opd, tau, s)) != hipSuccess) return hip_fail(e, "osog_render_multi: raster");
  if ((e = launch_pass1(u, opd, tau, b, ctx->twiddle, s)) != hipSuccess)
    return hip_fail(e, "osog_render_multi: pass 1");
  // passes 2 and 3 per mode, one after the other in the second band buffer
  for (int m = 0; m < n_modes; ++m) {
    FrameBufs bm = b;
    bm.band = b.band2;
    if (plans[m].kx_n > 0 &&
        (e = launch_pass2(plans[m], globals + 4 * m, bm, ctx->twiddle, s, b.band, u.kx_lo, u.kx_n)) != hipSuccess)
      return hip_fail(e, "osog_render_multi: pass 2");
    if ((e = launch_pass3(plans[m], bm, ctx->twiddle, intensity_out[m], s)) != hipSuccess)
      return hip_fail(e, "osog_render_multi: pass 3");
  }
  return OSOG_OK;
}

osog_status osog_render_backward(osog_context* ctx, void* stream, int32_t height, int32_t width,
                                 const float* soa, int64_t n, int64_t ld, const osog_optics* optics,
                                 const float* globals, const float* grad_intensity,
                                 const float* grad_opd, float* grad_soa, float* grad_globals,
                                 void* workspace, size_t workspace_bytes) {
  osog_status st = check_frame(ctx, height, width, soa, n, ld, optics, globals);
  if (st != OSOG_OK) return st;
  if (optics->mode == OSOG_DIC_INCOHERENT)
    return fail(OSOG_ERR_UNSUPPORTED, "osog_render_backward: the incoherent DIC has no adjoint");
  if (!grad_intensity) return fail(OSOG_ERR_INVALID_ARGUMENT, "grad_intensity is NULL");
  if (!workspace) return fail(OSOG_ERR_WORKSPACE, "workspace is NULL");
  int ppp = 0;
  for (int cand = 1 << 20; cand >= 1; cand >>= 1)
    if (frame_workspace_bytes(height, width, n, tile_of(ctx, height, width, 0), tile_of(ctx, height, width, 1), cand, true) <= workspace_bytes) {
      ppp = cand;
      break;
    }
  if (ppp == 0) return fail(OSOG_ERR_WORKSPACE, "workspace smaller than osog_workspace_size(with_backward=1)");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  int64_t cap = 0;
  FrameBufs b = carve(workspace, height, width, n, tile_of(ctx, height, width, 0), tile_of(ctx, height, width, 1), ppp, true, &cap);
  FramePlan p = make_plan(ctx, height, width, n, ld, *optics, cap);
  hipStream_t s = (hipStream_t)stream;
  Profiler* pr = ctx->prof;
  const float2* tw = ctx->twiddle;
  // recompute the forward intermediates: OPD, row spectra A (band), B = IDFT_y(U~ H) (band2)
  profile_begin(pr, OSOG_STAGE_BINNING, s);
  if ((e = launch_binning(p, soa, b, s)) != hipSuccess) return hip_fail(e, "backward: binning");
  profile_end(pr, OSOG_STAGE_BINNING, s);
  profile_begin(pr, OSOG_STAGE_RASTER, s);
  if ((e = launch_raster(p, b, b.opd, b.tau, s)) != hipSuccess) return hip_fail(e, "backward: raster");
  profile_end(pr, OSOG_STAGE_RASTER, s);
  profile_begin(pr, OSOG_STAGE_PASS1, s);
  if ((e = launch_pass1(p, b.opd, b.tau, b, tw, s)) != hipSuccess) return hip_fail(e, "backward: pass 1");
  profile_end(pr, OSOG_STAGE_PASS1, s);
  if (p.kx_n > 0) {
    profile_begin(pr, OSOG_STAGE_PASS2, s);
    if ((e = launch_pass2_keep(p, globals, b, tw, s)) != hipSuccess) return hip_fail(e, "backward: pass 2");
    profile_end(pr, OSOG_STAGE_PASS2, s);
    profile_begin(pr, OSOG_STAGE_ADJ_PASS3, s);
    if ((e = launch_adj_pass3(p, b, tw, grad_intensity, s)) != hipSuccess) return hip_fail(e, "backward: adj pass 3");
    profile_end(pr, OSOG_STAGE_ADJ_PASS3, s);
    profile_begin(pr, OSOG_STAGE_ADJ_PASS2, s);
    if ((e = launch_adj_pass2(p, globals, b, tw, s)) != hipSuccess) return hip_fail(e, "backward: adj pass 2");
    profile_end(pr, OSOG_STAGE_ADJ_PASS2, s);
  }
  profile_begin(pr, OSOG_STAGE_ADJ_PASS1, s);
  if ((e = launch_adj_pass1(p, b.opd, b.tau, grad_opd, b, tw, s)) != hipSuccess)
    return hip_fail(e, "backward: adj pass 1");
  profile_end(pr, OSOG_STAGE_ADJ_PASS1, s);
  if (grad_soa) {
    profile_begin(pr, OSOG_STAGE_ADJ_RASTER, s);
    if ((e = launch_raster_adjoint(p, soa, b, grad_soa, s)) != hipSuccess) return hip_fail(e, "backward: raster adjoint");
    profile_end(pr, OSOG_STAGE_ADJ_RASTER, s);
  }
  if (grad_globals && (e = launch_global_grads(p, b, grad_globals, s)) != hipSuccess)
    return hip_fail(e, "backward: global gradients");
  return OSOG_OK;
}

osog_status osog_set_habits(osog_context* ctx, int32_t n_habits, const int32_t* face_counts, const float* faces,
                            const float* radius, const float* topo_amplitude_um, const float* topo_cell_px,
                            uint64_t topo_seed) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (n_habits < 0 || n_habits > kMaxHabits)
    return fail(OSOG_ERR_INVALID_ARGUMENT, "n_habits must be in [0, 64]");
  if (n_habits > 0 && (!face_counts || !faces || !radius || !topo_amplitude_um || !topo_cell_px))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "habit arrays are NULL");
  std::vector<float4> tab(3 * kMaxHabits * kMaxFaces + 0, make_float4(0.f, 0.f, 0.f, 0.f));
  float4* enc = tab.data();
  float4* raw = enc + kMaxHabits * kMaxFaces;
  float4* info = raw + kMaxHabits * kMaxFaces;
  int64_t off = 0;
  for (int k = 0; k < n_habits; ++k) {
    const int m = face_counts[k];
    const std::string hk = "habit " + std::to_string(k) + ": ";
    if (m < 4 || m > kMaxFaces) return fail(OSOG_ERR_INVALID_ARGUMENT, hk + "needs 4..32 faces");
    const float* f = faces + 4 * off;
    for (int q = 0; q < 4 * m; ++q)
      if (!std::isfinite(f[q])) return fail(OSOG_ERR_INVALID_ARGUMENT, hk + "faces must be finite");
    double max_r = 0.0;
    bool bounded = true;
    if (!habit_vertices(f, m, &max_r, &bounded)) return fail(OSOG_ERR_INVALID_ARGUMENT, hk + "empty polytope");
    if (!bounded) return fail(OSOG_ERR_INVALID_ARGUMENT, hk + "unbounded polytope");
    if (!(radius[k] >= max_r * (1.0 - 1e-6)) || !std::isfinite(radius[k]))
      return fail(OSOG_ERR_INVALID_ARGUMENT, hk + "radius must bound sqrt(U^2 + V^2) over the polytope (" +
                                                 std::to_string(max_r) + ")");
    const float amp = topo_amplitude_um[k], cell = topo_cell_px[k];
    if (!(amp >= 0.0f) || !std::isfinite(amp))
      return fail(OSOG_ERR_INVALID_ARGUMENT, hk + "topography amplitude must be finite and >= 0");
    const int ci = (int)cell;
    if (!((float)ci == cell && pow2_in(ci, 1, 256)))
      return fail(OSOG_ERR_INVALID_ARGUMENT, hk + "topography cell must be a power of two in [1, 256] px");
    for (int q = 0; q < m; ++q) {
      const float nx = f[4 * q], ny = f[4 * q + 1], nz = f[4 * q + 2], d = f[4 * q + 3];
      raw[k * kMaxFaces + q] = make_float4(nx, ny, nz, d);
      if (nz != 0.0f)  // W bound (d - nx U - ny V) / nz, upper for nz > 0, lower for nz < 0
        enc[k * kMaxFaces + q] = make_float4(-nx / nz, -ny / nz, d / nz, nz > 0.0f ? 1.0f : -1.0f);
      else
        enc[k * kMaxFaces + q] = make_float4(nx, ny, -d, 0.0f);
    }
    info[k] = make_float4((float)m, radius[k], amp, cell);
    off += m;
  }
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  // work already queued may still read the old table
  if ((e = hipDeviceSynchronize()) != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  if (!ctx->hab && (e = hipMalloc(&ctx->hab, sizeof(float4) * tab.size())) != hipSuccess) {
    ctx->hab = nullptr;
    return hip_fail(e, "hipMalloc(habits)");
  }
  if ((e = hipMemcpy(ctx->hab, tab.data(), sizeof(float4) * tab.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return hip_fail(e, "hipMemcpy(habits)");
  ctx->n_habits = n_habits;
  ctx->topo_seed = topo_seed;
  ctx->habit_gen++;
  return OSOG_OK;
}

osog_status osog_spectral_workspace_size(int32_t height, int32_t width, size_t* bytes) {
  if (!bytes) return fail(OSOG_ERR_INVALID_ARGUMENT, "bytes is NULL");
  if (!pow2_in(height, 32, 4096) || !pow2_in(width, 32, 4096))
    return fail(OSOG_ERR_UNSUPPORTED, "height and width must be powers of two in [32, 4096]");
  *bytes = spectral_workspace_bytes(height, width);
  return OSOG_OK;
}

static osog_status spectral_check(osog_context* ctx, int32_t height, int32_t width, float eps, void* workspace,
                                  size_t workspace_bytes) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (!pow2_in(height, 32, 4096) || !pow2_in(width, 32, 4096))
    return fail(OSOG_ERR_UNSUPPORTED, "height and width must be powers of two in [32, 4096]");
  if (!(eps > 0.0f) || !std::isfinite(eps)) return fail(OSOG_ERR_INVALID_ARGUMENT, "eps must be finite and > 0");
  if (!workspace || workspace_bytes < spectral_workspace_bytes(height, width))
    return fail(OSOG_ERR_WORKSPACE, "workspace smaller than osog_spectral_workspace_size()");
  return OSOG_OK;
}

osog_status osog_spectral_target(osog_context* ctx, void* stream, int32_t height, int32_t width,
                                 const float* target, float eps, float* target_logamp, void* workspace,
                                 size_t workspace_bytes) {
  osog_status st = spectral_check(ctx, height, width, eps, workspace, workspace_bytes);
  if (st != OSOG_OK) return st;
  if (!target || !target_logamp) return fail(OSOG_ERR_INVALID_ARGUMENT, "target or target_logamp is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  e = spectral_run(height, width, target, nullptr, target_logamp, eps, nullptr, nullptr, workspace, ctx->twiddle,
                   (hipStream_t)stream);
  return e == hipSuccess ? OSOG_OK : hip_fail(e, "osog_spectral_target launch");
}

osog_status osog_spectral_loss(osog_context* ctx, void* stream, int32_t height, int32_t width,
                               const float* image, const float* target_logamp, float eps, float* loss_out,
                               float* grad_out, void* workspace, size_t workspace_bytes) {
  osog_status st = spectral_check(ctx, height, width, eps, workspace, workspace_bytes);
  if (st != OSOG_OK) return st;
  if (!image || !target_logamp || !loss_out)
    return fail(OSOG_ERR_INVALID_ARGUMENT, "image, target_logamp or loss_out is NULL");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  e = spectral_run(height, width, image, target_logamp, nullptr, eps, loss_out, grad_out, workspace, ctx->twiddle,
                   (hipStream_t)stream);
  return e == hipSuccess ? OSOG_OK : hip_fail(e, "osog_spectral_loss launch");
}

osog_status osog_bin(osog_context* ctx, void* stream, int32_t height, int32_t width,
                     const float* soa, int64_t n, int64_t ld, int32_t* keys_out, int32_t* pids_out,
                     int64_t capacity, int32_t* pair_count_out, int32_t* tile_start_out,
                     int32_t* counts_out, void* workspace, size_t workspace_bytes) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (n < 0 || n > INT_MAX || ld < n) return fail(OSOG_ERR_INVALID_ARGUMENT, "bad n or ld");
  if (n > 0 && !soa) return fail(OSOG_ERR_INVALID_ARGUMENT, "soa is NULL");
  if (!keys_out || !pids_out || !pair_count_out || !tile_start_out)
    return fail(OSOG_ERR_INVALID_ARGUMENT, "output pointer is NULL");
  if (capacity < 0 || capacity > INT_MAX - 1) return fail(OSOG_ERR_INVALID_ARGUMENT, "bad capacity");
  if (!pow2_in(height, 32, 4096) || !pow2_in(width, 32, 4096))
    return fail(OSOG_ERR_UNSUPPORTED, "height and width must be powers of two in [32, 4096]");
  if (height % tile_of(ctx, height, width, 0) || width % tile_of(ctx, height, width, 1))
    return fail(OSOG_ERR_UNSUPPORTED, "canvas sides must be multiples of the tile sides");
  size_t need = frame_workspace_bytes(height, width, n, tile_of(ctx, height, width, 0), tile_of(ctx, height, width, 1), 1, false);
  if (!workspace || workspace_bytes < need) return fail(OSOG_ERR_WORKSPACE, "workspace too small");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  int ppp = 1;
  for (int cand = 1 << 20; cand >= 1; cand >>= 1)
    if (frame_workspace_bytes(height, width, n, tile_of(ctx, height, width, 0), tile_of(ctx, height, width, 1), cand, false) <= workspace_bytes) {
      ppp = cand;
      break;
    }
  int64_t cap = 0;
  FrameBufs b = carve(workspace, height, width, n, tile_of(ctx, height, width, 0), tile_of(ctx, height, width, 1), ppp, false, &cap);
  osog_optics o{};
  o.mode = OSOG_BRIGHTFIELD; o.wavelength_um = 0.55; o.na = 0.5; o.n_medium = 1.33; o.pixel_um = 0.1;
  FramePlan p = make_plan(ctx, height, width, n, ld, o, cap);
  hipStream_t s = (hipStream_t)stream;
  if ((e = launch_binning(p, soa, b, s)) != hipSuccess) return hip_fail(e, "osog_bin launch");
  if ((e = launch_bin_outputs(p, b, keys_out, pids_out, capacity, tile_start_out, s)) != hipSuccess)
    return hip_fail(e, "osog_bin sort");
  if ((e = hipMemcpyAsync(pair_count_out, b.scal + 3, sizeof(int32_t), hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(e, "copy pair count");
  if (counts_out && n > 0 &&
      (e = hipMemcpyAsync(counts_out, b.counts, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s)) != hipSuccess)
    return hip_fail(e, "copy counts");
  return OSOG_OK;
}

osog_status osog_band_info(const osog_context* ctx, int32_t height, int32_t width,
                           const osog_optics* optics, int32_t* kx_lo, int32_t* kx_n) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (!kx_lo || !kx_n) return fail(OSOG_ERR_INVALID_ARGUMENT, "output pointer is NULL");
  osog_status st = check_optics(optics);
  if (st != OSOG_OK) return st;
  if (!pow2_in(height, 32, 4096) || !pow2_in(width, 32, 4096))
    return fail(OSOG_ERR_UNSUPPORTED, "height and width must be powers of two in [32, 4096]");
  int lo = 0, nn = 0;
  band_range(height, width, *optics, &lo, &nn);
  *kx_lo = lo;
  *kx_n = nn;
  return OSOG_OK;
}

static osog_status check_batch(osog_context* ctx, const osog_frame* frames, int32_t n_frames) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (n_frames <= 0 || !frames) return fail(OSOG_ERR_INVALID_ARGUMENT, "need n_frames >= 1 and a frame array");
  for (int f = 0; f < n_frames; ++f) {
    const osog_frame& fr = frames[f];
    int th, tw;
    context_tiling(ctx, fr.height, fr.width, &th, &tw);
    osog_status st = check_optics(&fr.optics);
    if (st != OSOG_OK) return fail(st, "frame " + std::to_string(f) + ": " + g_last_error);
    if (fr.n < 0 || fr.n > INT_MAX || fr.ld < fr.n || (fr.n > 0 && !fr.soa) || !fr.globals || !fr.intensity_out)
      return fail(OSOG_ERR_INVALID_ARGUMENT, "frame " + std::to_string(f) + ": bad n/ld or NULL pointer");
    if (!pow2_in(fr.height, 32, 4096) || !pow2_in(fr.width, 32, 4096) || fr.height % th || fr.width % tw)
      return fail(OSOG_ERR_UNSUPPORTED, "frame " + std::to_string(f) + ": canvas size not supported");
  }
  return OSOG_OK;
}

osog_status osog_batch_workspace_size(osog_context* ctx, const osog_frame* frames, int32_t n_frames,
                                      int32_t pairs_per_particle, size_t* bytes) {
  osog_status st = check_batch(ctx, frames, n_frames);
  if (st != OSOG_OK) return st;
  if (!bytes) return fail(OSOG_ERR_INVALID_ARGUMENT, "bytes is NULL");
  if (pairs_per_particle < 0) return fail(OSOG_ERR_INVALID_ARGUMENT, "pairs_per_particle must be >= 0");
  *bytes = batch_workspace_bytes(ctx, frames, n_frames, effective_ppp(pairs_per_particle));
  return OSOG_OK;
}

osog_status osog_batch_render(osog_context* ctx, void* stream, const osog_frame* frames, int32_t n_frames,
                              void* workspace, size_t workspace_bytes, uint64_t* frame_done_ns) {
  osog_status st = check_batch(ctx, frames, n_frames);
  if (st != OSOG_OK) return st;
  if (!workspace) return fail(OSOG_ERR_WORKSPACE, "workspace is NULL");
  int ppp = 0;
  for (int cand = 1 << 20; cand >= 1; cand >>= 1)
    if (batch_workspace_bytes(ctx, frames, n_frames, cand) <= workspace_bytes) { ppp = cand; break; }
  if (ppp == 0) return fail(OSOG_ERR_WORKSPACE, "workspace smaller than osog_batch_workspace_size()");
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  std::string err;
  Profiler* pr = ctx->prof;
  profile_begin(pr, OSOG_STAGE_BATCH, (hipStream_t)stream);
  e = batch_render(ctx, (hipStream_t)stream, frames, n_frames, ppp, ctx->batch_group, workspace,
                   workspace_bytes, frame_done_ns, &err);
  profile_end(pr, OSOG_STAGE_BATCH, (hipStream_t)stream);
  if (e != hipSuccess) return err.empty() ? hip_fail(e, "osog_batch_render") : fail(OSOG_ERR_WORKSPACE, err);
  return OSOG_OK;
}

osog_status osog_batch_error(osog_context* ctx, void* workspace, int32_t* flag) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (!workspace || !flag) return fail(OSOG_ERR_INVALID_ARGUMENT, "NULL pointer");
  hipError_t e = batch_error_flag(workspace, flag);
  if (e != hipSuccess) return hip_fail(e, "osog_batch_error");
  return OSOG_OK;
}

osog_status osog_set_batch_group(osog_context* ctx, int32_t group) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (group < 0) return fail(OSOG_ERR_INVALID_ARGUMENT, "group must be >= 0 (0: the maximum, 8)");
  ctx->batch_group = group;
  return OSOG_OK;
}

osog_status osog_set_size_tiling(osog_context* ctx, int32_t height, int32_t width, int32_t tile_h, int32_t tile_w) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (!tile_shape_ok(tile_h, tile_w) || !pow2_in(height, 32, 4096) || !pow2_in(width, 32, 4096) ||
      height % tile_h || width % tile_w)
    return fail(OSOG_ERR_UNSUPPORTED, "tiling must divide the canvas, powers of two, 256 <= tile_h * tile_w <= 1024");
  ctx->size_tiling[{height, width}] = {tile_h, tile_w};
  return OSOG_OK;
}

osog_status osog_cnn_param_count(int64_t* count) {
  if (!count) return fail(OSOG_ERR_INVALID_ARGUMENT, "count is NULL");
  *count = cnn_param_count();
  return OSOG_OK;
}

static osog_status check_cnn_shape(int32_t batch, int32_t height, int32_t width) {
  if (batch < 1 || height < 16 || width < 16 || height % 16 || width % 16 || height > 8192 || width > 8192)
    return fail(OSOG_ERR_UNSUPPORTED, "batch >= 1 and height, width multiples of 16 in [16, 8192]");
  if ((int64_t)batch * height * width > (int64_t)1 << 31)
    return fail(OSOG_ERR_UNSUPPORTED, "batch * height * width must stay below 2^31");
  return OSOG_OK;
}

osog_status osog_cnn_workspace_size(int32_t batch, int32_t height, int32_t width, size_t* bytes) {
  if (!bytes) return fail(OSOG_ERR_INVALID_ARGUMENT, "bytes is NULL");
  osog_status st = check_cnn_shape(batch, height, width);
  if (st != OSOG_OK) return st;
  *bytes = cnn_workspace_bytes(batch, height, width);
  return OSOG_OK;
}

osog_status osog_cnn_forward(osog_context* ctx, void* stream, int32_t batch, int32_t height, int32_t width,
                             const float* images, const float* params, float* pred, void* workspace,
                             size_t workspace_bytes) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  osog_status st = check_cnn_shape(batch, height, width);
  if (st != OSOG_OK) return st;
  if (!images || !params || !pred) return fail(OSOG_ERR_INVALID_ARGUMENT, "NULL pointer");
  if (!workspace || workspace_bytes < cnn_workspace_bytes(batch, height, width))
    return fail(OSOG_ERR_WORKSPACE, "workspace smaller than osog_cnn_workspace_size()");
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess) e = cnn_forward(batch, height, width, images, params, pred, workspace, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "osog_cnn_forward");
  return OSOG_OK;
}

osog_status osog_cnn_train_step(osog_context* ctx, void* stream, int32_t batch, int32_t height, int32_t width,
                                const float* images, const float* targets, float* params, float* m, float* v,
                                int32_t step, float lr, float* loss, float* grads_out, void* workspace,
                                size_t workspace_bytes) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  osog_status st = check_cnn_shape(batch, height, width);
  if (st != OSOG_OK) return st;
  if (!images || !targets || !params) return fail(OSOG_ERR_INVALID_ARGUMENT, "NULL pointer");
  if (step < 0 || (step > 0 && (!m || !v)) || !std::isfinite(lr))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "step >= 0 (with m, v when step > 0) and a finite lr");
  if (!workspace || workspace_bytes < cnn_workspace_bytes(batch, height, width))
    return fail(OSOG_ERR_WORKSPACE, "workspace smaller than osog_cnn_workspace_size()");
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess)
    e = cnn_train_step(batch, height, width, images, targets, params, m, v, step, lr, loss, grads_out, workspace,
                       (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "osog_cnn_train_step");
  return OSOG_OK;
}

static osog_status check_conv(int32_t mode, int32_t batch, int32_t height, int32_t width, int32_t c_in,
                              int32_t c_out, int32_t stride) {
  if (mode < 0 || mode > 2) return fail(OSOG_ERR_INVALID_ARGUMENT, "mode must be 0, 1 or 2");
  if (batch < 1 || height < 2 || width < 2 || c_in < 1 || c_out < 1 || (stride != 1 && stride != 2) ||
      (stride == 2 && (height % 2 || width % 2)))
    return fail(OSOG_ERR_INVALID_ARGUMENT, "bad convolution shape");
  if ((int64_t)batch * height * width * std::max(c_in, c_out) > (int64_t)1 << 31)
    return fail(OSOG_ERR_UNSUPPORTED, "convolution too large");
  return OSOG_OK;
}

osog_status osog_conv3x3_workspace_size(int32_t mode, int32_t batch, int32_t height, int32_t width,
                                        int32_t c_in, int32_t c_out, int32_t stride, size_t* bytes) {
  if (!bytes) return fail(OSOG_ERR_INVALID_ARGUMENT, "bytes is NULL");
  osog_status st = check_conv(mode, batch, height, width, c_in, c_out, stride);
  if (st != OSOG_OK) return st;
  *bytes = conv3x3_workspace_bytes(mode, batch, height, width, c_in, c_out, stride);
  return OSOG_OK;
}

osog_status osog_conv3x3(osog_context* ctx, void* stream, int32_t mode, int32_t batch, int32_t height,
                         int32_t width, int32_t c_in, int32_t c_out, int32_t stride, const uint16_t* x,
                         const uint16_t* y, const uint16_t* grad_y, const uint16_t* w, const float* bias,
                         uint16_t* out_bf16, float* out_f32, void* workspace, size_t workspace_bytes) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  osog_status st = check_conv(mode, batch, height, width, c_in, c_out, stride);
  if (st != OSOG_OK) return st;
  const bool ok = mode == 0 ? (x && w && bias && out_bf16)
                : mode == 1 ? (y && grad_y && w && out_bf16) : (x && y && grad_y && out_f32);
  if (!ok) return fail(OSOG_ERR_INVALID_ARGUMENT, "NULL pointer");
  if (!workspace || workspace_bytes < conv3x3_workspace_bytes(mode, batch, height, width, c_in, c_out, stride))
    return fail(OSOG_ERR_WORKSPACE, "workspace smaller than osog_conv3x3_workspace_size()");
  hipError_t e = hipSetDevice(ctx->device);
  if (e == hipSuccess)
    e = conv3x3(mode, batch, height, width, c_in, c_out, stride, x, y, grad_y, w, bias, out_bf16, out_f32, workspace,
                (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "osog_conv3x3");
  return OSOG_OK;
}

osog_status osog_set_size_radix(osog_context* ctx, int32_t height, int32_t width, int32_t fft_radix) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (fft_radix != 4 && fft_radix != 8) return fail(OSOG_ERR_UNSUPPORTED, "fft_radix must be 4 or 8");
  if (!pow2_in(height, 32, 4096) || !pow2_in(width, 32, 4096))
    return fail(OSOG_ERR_UNSUPPORTED, "height and width must be powers of two in [32, 4096]");
  ctx->size_radix[{height, width}] = fft_radix;
  return OSOG_OK;
}

osog_status osog_autotune(osog_context* ctx, void* stream, int32_t height, int32_t width, const float* soa,
                          int64_t n, int64_t ld, const osog_optics* optics, const float* globals,
                          float* intensity_out, void* workspace, size_t workspace_bytes, int32_t reps,
                          int32_t* tile_h, int32_t* tile_w, int32_t* fft_radix, float* best_ms) {
  osog_status st = check_frame(ctx, height, width, soa, n, ld, optics, globals);
  if (st != OSOG_OK) return st;
  if (!intensity_out || !tile_h || !tile_w || !fft_radix || reps < 1)
    return fail(OSOG_ERR_INVALID_ARGUMENT, "NULL output or reps < 1");
  hipStream_t s = (hipStream_t)stream;
  const std::pair<int, int> key{height, width};
  const auto saved_t = ctx->size_tiling.find(key) != ctx->size_tiling.end()
                           ? std::optional<std::pair<int, int>>(ctx->size_tiling[key]) : std::nullopt;
  const auto saved_r = ctx->size_radix.find(key) != ctx->size_radix.end()
                           ? std::optional<int>(ctx->size_radix[key]) : std::nullopt;
  const int cand_t[][2] = {{16, 16}, {32, 32}, {32, 16}, {16, 32}, {64, 16}};
  constexpr int n_cand_t = (int)(sizeof(cand_t) / sizeof(cand_t[0]));
  const int cand_r[2] = {8, 4};
  float best = 1e30f;
  int bt = -1, br = -1;
  hipEvent_t e0, e1;
  hipError_t e = hipSetDevice(ctx->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  if ((e = hipEventCreate(&e0)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  if ((e = hipEventCreate(&e1)) != hipSuccess) { (void)hipEventDestroy(e0); return hip_fail(e, "hipEventCreate"); }
  osog_status out = OSOG_OK;
  for (int ti = 0; ti < n_cand_t && out == OSOG_OK; ++ti) {
    if (height % cand_t[ti][0] || width % cand_t[ti][1]) continue;
    for (int ri = 0; ri < 2 && out == OSOG_OK; ++ri) {
      ctx->size_tiling[key] = {cand_t[ti][0], cand_t[ti][1]};
      ctx->size_radix[key] = cand_r[ri];
      out = osog_render(ctx, stream, height, width, soa, n, ld, optics, globals, nullptr, intensity_out,
                        workspace, workspace_bytes);
      if (out != OSOG_OK) break;
      (void)hipEventRecord(e0, s);
      for (int r = 0; r < reps && out == OSOG_OK; ++r)
        out = osog_render(ctx, stream, height, width, soa, n, ld, optics, globals, nullptr, intensity_out,
                          workspace, workspace_bytes);
      (void)hipEventRecord(e1, s);
      if ((e = hipEventSynchronize(e1)) != hipSuccess) { out = hip_fail(e, "autotune timing"); break; }
      float ms = 0.0f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      ms /= (float)reps;
      if (ms < best) { best = ms; bt = ti; br = ri; }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (out != OSOG_OK || bt < 0) {
    if (saved_t) ctx->size_tiling[key] = *saved_t; else ctx->size_tiling.erase(key);
    if (saved_r) ctx->size_radix[key] = *saved_r; else ctx->size_radix.erase(key);
    return out != OSOG_OK ? out : fail(OSOG_ERR_UNSUPPORTED, "no candidate tiling divides the canvas");
  }
  ctx->size_tiling[key] = {cand_t[bt][0], cand_t[bt][1]};
  ctx->size_radix[key] = cand_r[br];
  *tile_h = cand_t[bt][0];
  *tile_w = cand_t[bt][1];
  *fft_radix = cand_r[br];
  if (best_ms) *best_ms = best;
  return OSOG_OK;
}

osog_status osog_philox4x32_10(void* stream, const uint32_t* ctr, int64_t count, uint32_t key0,
                               uint32_t key1, uint32_t* out) {
  if (count < 0) return fail(OSOG_ERR_INVALID_ARGUMENT, "count must be >= 0");
  if (count > 0 && (!ctr || !out)) return fail(OSOG_ERR_INVALID_ARGUMENT, "NULL pointer");
  if (count == 0) return OSOG_OK;
  hipError_t e = launch_philox(ctr, count, key0, key1, out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "osog_philox4x32_10 launch");
  return OSOG_OK;
}

osog_status osog_profile_enable(osog_context* ctx, int32_t enable) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  profiler_set(ctx->prof, enable != 0);
  return OSOG_OK;
}

osog_status osog_profile_read(osog_context* ctx, double* ms, int64_t* launches) {
  if (!ctx) return fail(OSOG_ERR_NOT_INITIALIZED, "context is NULL");
  if (!ms || !launches) return fail(OSOG_ERR_INVALID_ARGUMENT, "output pointer is NULL");
  hipError_t e = profiler_read(ctx->prof, ms, launches);
  if (e != hipSuccess) return hip_fail(e, "osog_profile_read");
  return OSOG_OK;
}

const char* osog_status_string(osog_status s) {
  switch (s) {
    case OSOG_OK: return "OSOG_OK";
    case OSOG_ERR_INVALID_ARGUMENT: return "OSOG_ERR_INVALID_ARGUMENT";
    case OSOG_ERR_UNSUPPORTED: return "OSOG_ERR_UNSUPPORTED";
    case OSOG_ERR_WORKSPACE: return "OSOG_ERR_WORKSPACE";
    case OSOG_ERR_HIP: return "OSOG_ERR_HIP";
    case OSOG_ERR_NOT_INITIALIZED: return "OSOG_ERR_NOT_INITIALIZED";
  }
  return "unknown osog_status";
}

const char* osog_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
