// Stage profiler: pairs of HIP events recorded on the launch stream around each
// stage, read back (and released) on request.
#include <hip/hip_runtime.h>

#include <vector>

#include "osog.h"
#include "osog_internal.h"

namespace osog {

struct Profiler {
  bool on = false;
  struct Rec { int stage; hipEvent_t a, b; };
  std::vector<Rec> recs;
  hipEvent_t open[OSOG_NSTAGES] = {};
};

Profiler* profiler_create() { return new Profiler(); }

static void release(Profiler* p) {
  for (auto& r : p->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  p->recs.clear();
  for (auto& e : p->open)
    if (e) { (void)hipEventDestroy(e); e = nullptr; }
}

void profiler_destroy(Profiler* p) {
  if (!p) return;
  release(p);
  delete p;
}

void profiler_set(Profiler* p, bool on) { p->on = on; }

void profile_begin(Profiler* p, int stage, hipStream_t s) {
  if (!p || !p->on) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  if (p->open[stage]) (void)hipEventDestroy(p->open[stage]);
  p->open[stage] = e;
}

void profile_end(Profiler* p, int stage, hipStream_t s) {
  if (!p || !p->on || !p->open[stage]) return;
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return;
  (void)hipEventRecord(e, s);
  p->recs.push_back({stage, p->open[stage], e});
  p->open[stage] = nullptr;
}

hipError_t profiler_read(Profiler* p, double* ms, int64_t* launches) {
  for (int k = 0; k < OSOG_NSTAGES; ++k) { ms[k] = 0.0; launches[k] = 0; }
  hipError_t err = hipSuccess;
  for (auto& r : p->recs) {
    hipError_t e = hipEventSynchronize(r.b);
    float t = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&t, r.a, r.b);
    if (e != hipSuccess) { err = e; continue; }
    ms[r.stage] += t;
    launches[r.stage] += 1;
  }
  release(p);
  return err;
}

}  // namespace osog
