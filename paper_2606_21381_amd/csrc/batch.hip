// Batched rendering of many frames of uneven size and particle count as ONE
// HIP graph launch, captured once per batch signature and replayed.
//
// Graph shape: a start node (clears the batch flags and stamps the launch
// time), then `branches` independent chains, frame f on chain f mod branches,
// each frame the same kernel sequence osog_render launches (binning, raster,
// three FFT passes with the noise fused into the last), followed by a one-thread
// node that stamps the frame's completion time and counts a pair-list overflow;
// the chains join at the end.  Frames on different chains run concurrently on
// the device's hardware queues, so small frames overlap large ones.  Every
// dependency is a graph edge: no workgroup ever waits for another.
//
// Kernel arguments (frame pointers, sizes, optics, the habit count and
// topography seed) and the raster build are fixed at capture, so the signature
// is the raw frame descriptors plus the workspace, the timestamp buffer, the
// per-size tiling and FFT radix, the branch count and the context's habit
// generation (which osog_set_habits advances).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "batch.h"
#include "osog_internal.h"
#include "stages.h"

namespace osog {

constexpr int kMaxBranches = 8;
constexpr int kBatchCtl = 64;  // ints at the head of the workspace: [1] = frames that overflowed

__global__ void __launch_bounds__(kThreads) k_batch_start(int* __restrict__ ctl,
                                                          unsigned long long* __restrict__ done, int nf,
                                                          double ns_per_tick) {
  const int t = threadIdx.x;
  if (t < kBatchCtl) ctl[t] = 0;
  if (t == 0 && done) done[nf] = (unsigned long long)((double)wall_clock64() * ns_per_tick);
}

__global__ void k_batch_stamp(unsigned long long* __restrict__ done, int f, const int* __restrict__ scal,
                              int* __restrict__ ctl, double ns_per_tick) {
  if (threadIdx.x != 0) return;
  if (scal[1]) atomicAdd(&ctl[1], 1);
  if (done) done[f] = (unsigned long long)((double)wall_clock64() * ns_per_tick);
}

// ---- host --------------------------------------------------------------------------
struct BatchEntry {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

struct BatchCache {
  std::map<std::string, BatchEntry> entries;
  hipStream_t capture = nullptr;
  hipStream_t branch[kMaxBranches] = {};
  hipEvent_t fork = nullptr;
  hipEvent_t join[kMaxBranches] = {};
};

BatchCache* batch_cache_create() { return new BatchCache(); }

void batch_cache_destroy(BatchCache* c) {
  if (!c) return;
  for (auto& kv : c->entries) {
    if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
    if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
  }
  for (int b = 0; b < kMaxBranches; ++b) {
    if (c->branch[b]) (void)hipStreamDestroy(c->branch[b]);
    if (c->join[b]) (void)hipEventDestroy(c->join[b]);
  }
  if (c->fork) (void)hipEventDestroy(c->fork);
  if (c->capture) (void)hipStreamDestroy(c->capture);
  delete c;
}

static size_t al(size_t v) { return (v + 255) & ~size_t(255); }

void context_tiling(const osog_context* ctx, int H, int W, int* th, int* tw);
int context_radix(const osog_context* ctx, int H, int W);
int context_device(const osog_context* ctx);
BatchCache* context_batch(osog_context* ctx);
uint64_t context_habit_generation(const osog_context* ctx);

// Workspace: the flags, then each frame's single-frame workspace.
static std::vector<size_t> batch_offsets(const osog_context* ctx, const osog_frame* frames, int nf, int ppp,
                                         size_t* total) {
  std::vector<size_t> off(nf);
  size_t o = al(sizeof(int) * kBatchCtl);
  for (int f = 0; f < nf; ++f) {
    int th, tw;
    context_tiling(ctx, frames[f].height, frames[f].width, &th, &tw);
    off[f] = o;
    // an incoherent DIC frame takes the larger carve (its spectra buffers)
    o += al(frame_workspace_bytes(frames[f].height, frames[f].width, frames[f].n, th, tw, ppp,
                                  frames[f].optics.mode == OSOG_DIC_INCOHERENT));
  }
  *total = o;
  return off;
}

size_t batch_workspace_bytes(const osog_context* ctx, const osog_frame* frames, int nf, int ppp) {
  size_t total = 0;
  (void)batch_offsets(ctx, frames, nf, ppp, &total);
  return total;
}

static hipError_t ensure_streams(BatchCache* c) {
  hipError_t e;
  if (!c->capture && (e = hipStreamCreateWithFlags(&c->capture, hipStreamNonBlocking)) != hipSuccess) return e;
  if (!c->fork && (e = hipEventCreateWithFlags(&c->fork, hipEventDisableTiming)) != hipSuccess) return e;
  for (int b = 0; b < kMaxBranches; ++b) {
    if (!c->branch[b] && (e = hipStreamCreateWithFlags(&c->branch[b], hipStreamNonBlocking)) != hipSuccess) return e;
    if (!c->join[b] && (e = hipEventCreateWithFlags(&c->join[b], hipEventDisableTiming)) != hipSuccess) return e;
  }
  return hipSuccess;
}

// Records the batch into the capture stream (and the branch streams it forks to).
static hipError_t record_batch(osog_context* ctx, BatchCache* c, const osog_frame* frames, int nf, int ppp,
                               int branches, char* ws, const std::vector<size_t>& off, uint64_t* frame_done_ns,
                               double ns_per_tick) {
  int* ctl = reinterpret_cast<int*>(ws);
  unsigned long long* done = reinterpret_cast<unsigned long long*>(frame_done_ns);
  hipLaunchKernelGGL(k_batch_start, dim3(1), dim3(kThreads), 0, c->capture, ctl, done, nf, ns_per_tick);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(c->fork, c->capture)) != hipSuccess) return e;
  for (int b = 0; b < branches; ++b)
    if ((e = hipStreamWaitEvent(c->branch[b], c->fork, 0)) != hipSuccess) return e;
  for (int f = 0; f < nf; ++f) {
    const osog_frame& fr = frames[f];
    hipStream_t s = c->branch[f % branches];
    int th, tw;
    context_tiling(ctx, fr.height, fr.width, &th, &tw);
    int64_t cap = 0;
    FrameBufs bufs = carve(ws + off[f], fr.height, fr.width, fr.n, th, tw, ppp,
                           fr.optics.mode == OSOG_DIC_INCOHERENT, &cap);
    FramePlan p = make_plan(ctx, fr.height, fr.width, fr.n, fr.ld, fr.optics, cap);
    if ((e = forward_frame(ctx, p, fr.soa, fr.globals, bufs, fr.opd_out, fr.intensity_out, s, false)) != hipSuccess)
      return e;
    hipLaunchKernelGGL(k_batch_stamp, dim3(1), dim3(64), 0, s, done, f, bufs.scal, ctl, ns_per_tick);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  for (int b = 0; b < branches; ++b) {
    if ((e = hipEventRecord(c->join[b], c->branch[b])) != hipSuccess) return e;
    if ((e = hipStreamWaitEvent(c->capture, c->join[b], 0)) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t batch_render(osog_context* ctx, hipStream_t stream, const osog_frame* frames, int nf, int ppp,
                        int group, void* workspace, size_t ws_bytes, uint64_t* frame_done_ns,
                        std::string* err) {
  size_t total = 0;
  const std::vector<size_t> off = batch_offsets(ctx, frames, nf, ppp, &total);
  if (ws_bytes < total) { *err = "workspace smaller than osog_batch_workspace_size()"; return hipErrorInvalidValue; }
  const int branches = std::max(1, std::min({group > 0 ? group : kMaxBranches, kMaxBranches, nf}));
  // signature: everything the captured kernel arguments depend on
  std::string sig(reinterpret_cast<const char*>(frames), sizeof(osog_frame) * (size_t)nf);
  const void* extra[2] = {workspace, frame_done_ns};
  sig.append(reinterpret_cast<const char*>(extra), sizeof(extra));
  const uint64_t gen = context_habit_generation(ctx);
  sig.append(reinterpret_cast<const char*>(&gen), sizeof(gen));
  std::vector<int> ints = {ppp, branches};
  for (int f = 0; f < nf; ++f) {
    int th, tw;
    context_tiling(ctx, frames[f].height, frames[f].width, &th, &tw);
    ints.push_back(th);
    ints.push_back(tw);
    ints.push_back(context_radix(ctx, frames[f].height, frames[f].width));
  }
  sig.append(reinterpret_cast<const char*>(ints.data()), sizeof(int) * ints.size());

  BatchCache* c = context_batch(ctx);
  hipError_t e;
  auto it = c->entries.find(sig);
  if (it == c->entries.end()) {
    if ((e = ensure_streams(c)) != hipSuccess) return e;
    int rate_khz = 0;
    (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, context_device(ctx));
    const double ns_per_tick = rate_khz > 0 ? 1.0e6 / (double)rate_khz : 10.0;
    BatchEntry E;
    if ((e = hipStreamBeginCapture(c->capture, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    const hipError_t rec = record_batch(ctx, c, frames, nf, ppp, branches, static_cast<char*>(workspace), off,
                                        frame_done_ns, ns_per_tick);
    e = hipStreamEndCapture(c->capture, &E.graph);
    if (rec != hipSuccess) {
      if (E.graph) (void)hipGraphDestroy(E.graph);
      return rec;
    }
    if (e != hipSuccess) return e;
    if ((e = hipGraphInstantiate(&E.exec, E.graph, nullptr, nullptr, 0)) != hipSuccess) {
      (void)hipGraphDestroy(E.graph);
      return e;
    }
    it = c->entries.emplace(sig, E).first;
  }
  return hipGraphLaunch(it->second.exec, stream);
}

hipError_t batch_error_flag(void* workspace, int* flag) {
  return hipMemcpy(flag, reinterpret_cast<int*>(workspace) + 1, sizeof(int), hipMemcpyDeviceToHost);
}

}  // namespace osog
