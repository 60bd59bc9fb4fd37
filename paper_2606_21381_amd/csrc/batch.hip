// Batched rendering of many frames of uneven size and particle count in ONE
// persistent kernel launch, captured in a HIP graph per batch signature.
//
// Work model: every stage of every frame is a list of workgroup-sized items
// (the same bodies the single-frame kernels run, stages.h).  Items are laid out
// in a queue in dependency order -- frames in groups of `group` consecutive
// frames, stage-major inside a group -- and resident workgroups pop them with
// one atomic.  Before running item (f, s, k), a workgroup waits until every
// item of the frame's previous non-empty stage has finished; an item only ever
// waits for items earlier in the queue, which running workgroups already hold,
// so the queue always drains.  Waits are bounded in time on the device's
// constant-rate clock, and so is a workgroup's working life: past either limit
// the workgroup raises an error flag, after which every workgroup only drains
// the queue (pops items without waiting or working), so the launch always ends.
// Producers publish with a release fence before bumping a stage's completion
// counter; consumers acquire after observing it.
//
// The workgroup that completes a frame's last stage stamps the frame's
// completion time (the device's constant-rate clock, converted to ns).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "batch.h"
#include "osog_internal.h"
#include "stages.h"

namespace osog {

enum Stage {
  ST_PREPARE = 0, ST_EMIT, ST_OFF0, ST_SCAT0, ST_OFF1, ST_SCAT1, ST_RASTER, ST_PASS1, ST_PASS2,
  ST_PASS3, ST_COUNT
};
constexpr int kScatterItems = 64;     // workgroup items per scatter stage (each loops over slices)
constexpr double kWaitSeconds = 1.0;  // one dependency wait, then the error path
constexpr double kLifeSeconds = 4.0;  // a workgroup's working life, then the error path

struct Segment {
  int frame, stage, count;
  int dep, dep_need;  // completion counter to wait on (frame * ST_COUNT + stage) and its target, or -1
  int last;           // 1 if this is the frame's last non-empty stage
  int pad[2];
};

struct BatchHeader {
  unsigned long long* frame_done;  // caller's timestamps (or null)
  double ns_per_tick;
  unsigned long long wait_ticks;   // longest wait for one dependency (device clock ticks)
  unsigned long long life_ticks;   // longest a workgroup keeps doing work after it starts
  int n_frames, nseg, total;
  int pad;
};

// ---- the persistent kernel ------------------------------------------------------
__device__ __forceinline__ int find_segment(const int* __restrict__ seg_start, int nseg, int item) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (seg_start[mid] <= item) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int LOG, int MAXR>
__device__ __forceinline__ void run_fft_plan(const FrameDev& F, int stage, int k, const float2* tw, char* lds) {
  if (stage == ST_PASS1) pass1_body<LOG, MAXR>(F, k, tw, lds);
  else if (stage == ST_PASS2) pass2_body<LOG, MAXR>(F, k, tw, lds);
  else pass3_body<LOG, MAXR>(F, k, tw, lds);
}

template <int LOG>
__device__ __forceinline__ void run_fft_stage(const FrameDev& F, int stage, int k, const float2* tw, char* lds) {
  if (F.fft_radix == 4) run_fft_plan<LOG, 4>(F, stage, k, tw, lds);
  else run_fft_plan<LOG, 8>(F, stage, k, tw, lds);
}

__device__ __forceinline__ void fft_stage(const FrameDev& F, int stage, int k, const float2* tw, char* lds) {
  const int lg = stage == ST_PASS2 ? F.logH : F.logW;
  switch (lg) {
    case 5: run_fft_stage<5>(F, stage, k, tw, lds); break;
    case 6: run_fft_stage<6>(F, stage, k, tw, lds); break;
    case 7: run_fft_stage<7>(F, stage, k, tw, lds); break;
    case 8: run_fft_stage<8>(F, stage, k, tw, lds); break;
    case 9: run_fft_stage<9>(F, stage, k, tw, lds); break;
    case 10: run_fft_stage<10>(F, stage, k, tw, lds); break;
    case 11: run_fft_stage<11>(F, stage, k, tw, lds); break;
    default: run_fft_stage<12>(F, stage, k, tw, lds); break;
  }
}

__global__ void __launch_bounds__(kThreads) k_batch_clear(int* __restrict__ ctl, int n) {
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < n; i += gridDim.x * kThreads) ctl[i] = 0;
}

__global__ void __launch_bounds__(kThreads) k_batch(const BatchHeader* __restrict__ hdr,
                                                    const FrameDev* __restrict__ frames,
                                                    const int* __restrict__ seg_start,
                                                    const Segment* __restrict__ segs,
                                                    int* __restrict__ ctl,  // [0] queue head, [1] error
                                                    int* __restrict__ done,
                                                    const float2* __restrict__ tw) {
  __shared__ __align__(16) char lds[kStageLds];
  __shared__ int s_item, s_seg, s_skip;
  const int t = threadIdx.x;
  const int total = hdr->total, nseg = hdr->nseg;
  const unsigned long long born = wall_clock64();
  for (;;) {
    if (t == 0) {
      const int item = atomicAdd(&ctl[0], 1);
      s_item = item;
      s_skip = 0;
      if (item < total) {
        const int sg = find_segment(seg_start, nseg, item);
        s_seg = sg;
        if (item == 0 && hdr->frame_done)
          hdr->frame_done[hdr->n_frames] = (unsigned long long)((double)wall_clock64() * hdr->ns_per_tick);
        // After any error (here or in another workgroup) or past this workgroup's
        // working life, items are only drained: no wait, no work.
        bool bad = __hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                   wall_clock64() - born > hdr->life_ticks;
        // Wait for every item of the frame's previous non-empty stage.  The poll is
        // relaxed (no cache invalidation per iteration, which would stall the L2 of
        // this die for the producers); one acquire fence follows.  Bounded in time.
        const int dep = segs[sg].dep;
        if (!bad && dep >= 0) {
          const int need = segs[sg].dep_need;
          const unsigned long long w0 = wall_clock64();
          while (__hip_atomic_load(&done[dep], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
            __builtin_amdgcn_s_sleep(8);
            if (__hip_atomic_load(&ctl[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                wall_clock64() - w0 > hdr->wait_ticks) {
              bad = true;
              break;
            }
          }
        }
        if (bad) {
          atomicOr(&ctl[1], 1);
          s_skip = 1;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
    }
    __syncthreads();
    const int item = s_item;
    if (item >= total) break;
    const Segment sg = segs[s_seg];
    const int k = item - seg_start[s_seg];
    const FrameDev& F = frames[sg.frame];
    switch (s_skip ? -1 : sg.stage) {
      case ST_PREPARE: prepare_body(F, k, max(1, F.nblk), lds); break;
      case ST_EMIT: emit_body(F, k, lds); break;
      case ST_OFF0: digit_offsets_body(F, 0, k, lds); break;
      case ST_OFF1: digit_offsets_body(F, 1, k, lds); break;
      case ST_SCAT0:
      case ST_SCAT1: {
        const int P = F.scal[1] ? 0 : F.scal[0];
        const int nsl = (P + kThreads - 1) / kThreads;
        for (int sl = k; sl < nsl; sl += kScatterItems) scatter_body(F, sg.stage == ST_SCAT0 ? 0 : 1, sl, lds);
        break;
      }
      case ST_RASTER: {
        const int tile = 4 * k + (t >> 6);
        if (tile < F.n_tiles) raster_tile(F, tile, t & 63);
        break;
      }
      case ST_PASS1:
      case ST_PASS2:
      case ST_PASS3: fft_stage(F, sg.stage, k, tw, lds); break;
      default: break;
    }
    __syncthreads();
    if (t == 0) {
      __threadfence();
      const int prev = atomicAdd(&done[sg.frame * ST_COUNT + sg.stage], 1);
      if (prev + 1 == sg.count && sg.last && hdr->frame_done)
        hdr->frame_done[sg.frame] = (unsigned long long)((double)wall_clock64() * hdr->ns_per_tick);
    }
  }
}

// ---- host: planning, workspace layout, graph cache ------------------------------
struct BatchEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  void* host_buf = nullptr;  // pinned staging of the upload block
  size_t upload_bytes = 0;
  hipEvent_t done_ev = nullptr;
  bool in_flight = false;
};

struct BatchCache {
  std::map<std::string, BatchEntry> entries;
  hipStream_t capture = nullptr;
};

BatchCache* batch_cache_create() { return new BatchCache(); }

void batch_cache_destroy(BatchCache* c) {
  if (!c) return;
  for (auto& kv : c->entries) {
    BatchEntry& e = kv.second;
    if (e.done_ev) { (void)hipEventSynchronize(e.done_ev); (void)hipEventDestroy(e.done_ev); }
    if (e.exec) (void)hipGraphExecDestroy(e.exec);
    if (e.graph) (void)hipGraphDestroy(e.graph);
    if (e.host_buf) (void)hipHostFree(e.host_buf);
  }
  if (c->capture) (void)hipStreamDestroy(c->capture);
  delete c;
}

static size_t al(size_t v) { return (v + 255) & ~size_t(255); }

struct BatchLayout {
  size_t ctl_off, upload_off, upload_bytes, hdr_off, frames_off, segstart_off, segs_off, total;
  std::vector<size_t> frame_off, frame_bytes;
  int nctl;
};

static BatchLayout batch_layout(const std::vector<FramePlan>& plans, int ppp) {
  BatchLayout L;
  const int nf = (int)plans.size();
  const int max_seg = nf * ST_COUNT;
  L.nctl = 64 + nf * ST_COUNT;
  L.ctl_off = 0;
  size_t off = al(sizeof(int) * L.nctl);
  L.upload_off = off;
  L.hdr_off = 0;
  L.frames_off = al(sizeof(BatchHeader));
  L.segstart_off = L.frames_off + al(sizeof(FrameDev) * nf);
  L.segs_off = L.segstart_off + al(sizeof(int) * (max_seg + 1));
  L.upload_bytes = L.segs_off + al(sizeof(Segment) * (max_seg > 0 ? max_seg : 1));
  off += al(L.upload_bytes);
  for (const FramePlan& p : plans) {
    const size_t b = frame_workspace_bytes(p.H, p.W, p.n, p.tile_h, p.tile_w, ppp, false);
    L.frame_off.push_back(off);
    L.frame_bytes.push_back(b);
    off += al(b);
  }
  L.total = off;
  return L;
}

// Item counts per stage (0 = stage absent for this frame).
static void stage_counts(const FrameDev& F, int counts[ST_COUNT]) {
  const int nb = F.nblk;
  counts[ST_PREPARE] = nb > 0 ? nb : 1;
  counts[ST_EMIT] = nb > 0 ? nb : 1;
  const bool sort = F.d1 > 0 && nb > 0;
  counts[ST_OFF0] = sort ? (1 << F.d1) : 0;
  counts[ST_SCAT0] = sort ? kScatterItems : 0;
  counts[ST_OFF1] = sort && F.d2 > 0 ? (1 << F.d2) : 0;
  counts[ST_SCAT1] = sort && F.d2 > 0 ? kScatterItems : 0;
  counts[ST_RASTER] = (F.n_tiles + 3) / 4;
  counts[ST_PASS1] = F.H / F.o.rb;
  counts[ST_PASS2] = F.o.kx_n;
  counts[ST_PASS3] = F.H / F.o.rb;
}

FramePlan make_plan(const osog_context* ctx, int H, int W, int64_t n, int64_t ld, const osog_optics& o,
                    int64_t cap);
void context_tiling(const osog_context* ctx, int H, int W, int* th, int* tw);
int context_radix(const osog_context* ctx, int H, int W);
const float2* context_twiddle(const osog_context* ctx);
int context_device(const osog_context* ctx);
BatchCache* context_batch(osog_context* ctx);

static std::vector<FramePlan> batch_plans(const osog_context* ctx, const osog_frame* frames, int nf, int ppp) {
  std::vector<FramePlan> plans;
  for (int f = 0; f < nf; ++f) {
    const osog_frame& fr = frames[f];
    int th, tw;
    context_tiling(ctx, fr.height, fr.width, &th, &tw);
    FramePlan p = make_plan(ctx, fr.height, fr.width, fr.n, fr.ld, fr.optics, 0);
    p.tile_h = th; p.tile_w = tw;
    p.fft_radix = context_radix(ctx, fr.height, fr.width);
    p.ntx = fr.width / tw; p.nty = fr.height / th; p.n_tiles = p.ntx * p.nty;
    int kb = 0;
    while ((1 << kb) < p.n_tiles) ++kb;
    p.key_bits = kb;
    plans.push_back(p);
  }
  return plans;
}

size_t batch_workspace_bytes(const osog_context* ctx, const osog_frame* frames, int nf, int ppp) {
  return batch_layout(batch_plans(ctx, frames, nf, ppp), ppp).total;
}

hipError_t batch_render(osog_context* ctx, hipStream_t stream, const osog_frame* frames, int nf, int ppp,
                        int group, void* workspace, size_t ws_bytes, uint64_t* frame_done_ns,
                        std::string* err) {
  std::vector<FramePlan> plans = batch_plans(ctx, frames, nf, ppp);
  BatchLayout L = batch_layout(plans, ppp);
  if (ws_bytes < L.total) { *err = "workspace smaller than osog_batch_workspace_size()"; return hipErrorInvalidValue; }
  char* ws = static_cast<char*>(workspace);
  // device descriptors and the work queue
  std::vector<char> up(L.upload_bytes, 0);
  BatchHeader* hdr = reinterpret_cast<BatchHeader*>(up.data() + L.hdr_off);
  FrameDev* fd = reinterpret_cast<FrameDev*>(up.data() + L.frames_off);
  int* seg_start = reinterpret_cast<int*>(up.data() + L.segstart_off);
  Segment* segs = reinterpret_cast<Segment*>(up.data() + L.segs_off);
  std::vector<std::array<int, ST_COUNT>> counts(nf);
  std::string sig = std::to_string(nf) + ":" + std::to_string(ppp) + ":" + std::to_string(group) + ":" +
                    std::to_string((uintptr_t)workspace);
  for (int f = 0; f < nf; ++f) {
    FramePlan& p = plans[f];
    const size_t fb = L.frame_bytes[f];
    int64_t cap = 0;
    // the carve reproduces frame_workspace_bytes' layout at this frame's offset
    FrameBufs b = carve(ws + L.frame_off[f], p.H, p.W, p.n, p.tile_h, p.tile_w, ppp, false, &cap);
    (void)fb;
    p.cap = cap;
    FrameDev F = make_dev(p, b);
    F.soa = frames[f].soa;
    F.globals = frames[f].globals;
    F.opd = frames[f].opd_out ? frames[f].opd_out : b.opd;
    F.intensity = frames[f].intensity_out;
    fd[f] = F;
    stage_counts(F, counts[f].data());
    sig += "|" + std::to_string(p.H) + "," + std::to_string(p.W) + "," + std::to_string(p.n) + "," +
           std::to_string(p.tile_h) + "," + std::to_string(p.fft_radix) + "," + std::to_string(p.kx_lo) + "," + std::to_string(p.kx_n);
  }
  int nseg = 0, total = 0;
  std::vector<int> last_stage(nf, -1);
  for (int f = 0; f < nf; ++f)
    for (int st = 0; st < ST_COUNT; ++st)
      if (counts[f][st] > 0) last_stage[f] = st;
  const int g = group > 0 ? group : nf;
  for (int g0 = 0; g0 < nf; g0 += g)
    for (int st = 0; st < ST_COUNT; ++st)
      for (int f = g0; f < std::min(nf, g0 + g); ++f) {
        const int c = counts[f][st];
        if (c <= 0) continue;
        int dep = -1, need = 0;
        for (int q = st - 1; q >= 0; --q)
          if (counts[f][q] > 0) { dep = f * ST_COUNT + q; need = counts[f][q]; break; }
        Segment sgm{};
        sgm.frame = f; sgm.stage = st; sgm.count = c; sgm.dep = dep; sgm.dep_need = need;
        sgm.last = st == last_stage[f] ? 1 : 0;
        seg_start[nseg] = total;
        segs[nseg++] = sgm;
        total += c;
      }
  seg_start[nseg] = total;
  int rate_khz = 0;
  (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, context_device(ctx));
  hdr->frame_done = reinterpret_cast<unsigned long long*>(frame_done_ns);
  hdr->ns_per_tick = rate_khz > 0 ? 1.0e6 / (double)rate_khz : 10.0;
  const double ticks_per_s = rate_khz > 0 ? 1.0e3 * (double)rate_khz : 1.0e8;
  hdr->wait_ticks = (unsigned long long)(kWaitSeconds * ticks_per_s);
  hdr->life_ticks = (unsigned long long)(kLifeSeconds * ticks_per_s);
  hdr->n_frames = nf;
  hdr->nseg = nseg;
  hdr->total = total;

  BatchCache* cache = context_batch(ctx);
  hipError_t e;
  auto it = cache->entries.find(sig);
  if (it == cache->entries.end()) {
    BatchEntry E;
    E.upload_bytes = L.upload_bytes;
    if ((e = hipHostMalloc(&E.host_buf, L.upload_bytes, hipHostMallocDefault)) != hipSuccess) return e;
    if ((e = hipEventCreateWithFlags(&E.done_ev, hipEventDisableTiming)) != hipSuccess) return e;
    if (!cache->capture && (e = hipStreamCreateWithFlags(&cache->capture, hipStreamNonBlocking)) != hipSuccess)
      return e;
    int cus = 0;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, context_device(ctx));
    const int grid = std::max(1, std::min(total, 2 * std::max(cus, 1)));
    char* up_dev = ws + L.upload_off;
    int* ctl = reinterpret_cast<int*>(ws + L.ctl_off);
    int* done = ctl + 64;
    if ((e = hipStreamBeginCapture(cache->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    (void)hipMemcpyAsync(up_dev, E.host_buf, L.upload_bytes, hipMemcpyHostToDevice, cache->capture);
    hipLaunchKernelGGL(k_batch_clear, dim3(std::max(1, (L.nctl + kThreads - 1) / kThreads)), dim3(kThreads), 0,
                       cache->capture, ctl, L.nctl);
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(kThreads), 0, cache->capture,
                       reinterpret_cast<const BatchHeader*>(up_dev + L.hdr_off),
                       reinterpret_cast<const FrameDev*>(up_dev + L.frames_off),
                       reinterpret_cast<const int*>(up_dev + L.segstart_off),
                       reinterpret_cast<const Segment*>(up_dev + L.segs_off), ctl, done, context_twiddle(ctx));
    e = hipStreamEndCapture(cache->capture, &E.graph);
    if (e != hipSuccess) return e;
    if ((e = hipGraphInstantiate(&E.exec, E.graph, nullptr, nullptr, 0)) != hipSuccess) return e;
    it = cache->entries.emplace(sig, E).first;
  }
  BatchEntry& E = it->second;
  if (E.in_flight && (e = hipEventSynchronize(E.done_ev)) != hipSuccess) return e;
  std::memcpy(E.host_buf, up.data(), L.upload_bytes);
  if ((e = hipGraphLaunch(E.exec, stream)) != hipSuccess) return e;
  if ((e = hipEventRecord(E.done_ev, stream)) != hipSuccess) return e;
  E.in_flight = true;
  return hipSuccess;
}

hipError_t batch_error_flag(void* workspace, int* flag) {
  return hipMemcpy(flag, reinterpret_cast<int*>(workspace) + 1, sizeof(int), hipMemcpyDeviceToHost);
}

}  // namespace osog
