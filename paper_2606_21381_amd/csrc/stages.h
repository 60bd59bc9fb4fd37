// The forward renderer's stages as workgroup-level device bodies over a device
// frame descriptor.  The single-frame kernels (bin.hip, raster.hip, fft.hip)
// call these; the batch graph (batch.hip) replays those kernels, so a frame
// rendered alone or inside a batch goes through identical arithmetic.
//
// Every body is executed by one 256-thread workgroup (the raster body by one
// 64-lane wave) and receives a pointer to the LDS scratch its kernel declares
// (FFT buffers sized by fft_lds_f2); bodies that synchronise call
// __syncthreads() uniformly.
#pragma once

#include "bin_common.h"
#include "fft_common.h"
#include "geometry.h"
#include "osog_internal.h"

namespace osog {


// Everything a stage needs to know about one frame, in device-readable form.
struct FrameDev {
  int H, W, logH, logW, tile_h, tile_w, ntx, n_tiles;
  int fft_radix;                   // FFT plan: largest Stockham radix (8 or 4)
  int64_t n, ld, cap;              // cap: ids per tile bucket
  OpticsArgs o;
  float phase_k;
  const float* soa;
  const float* globals;
  float* opd;                      // caller's or workspace OPD canvas
  float* tau;                      // absorbance canvas (absorbing frames)
  float2* absr;                    // per particle (dmu * height, dmu) (absorbing frames)
  int absorb;
  const float4* hab_enc;           // polyhedral habits (see FramePlan)
  const float4* hab_raw;
  const float4* hab_info;
  int n_habits;
  uint32_t topo_lo, topo_hi;
  float* intensity;
  PRec* recs;
  int4* boxes;
  int* counts;                     // pairs per particle
  int* scal;                       // [1] tiles whose bucket overflowed, [3] total pairs (inspection)
  int* tile_count;                 // pairs per tile (the fill cursor; may exceed the bucket)
  int* tile_first;                 // inspection only: exclusive prefix of the tile counts
  int* pids;                       // n_tiles buckets of `cap` particle ids
  float2* band;
  double* colsum;
  // pass 2 reads its columns from band_in, whose in-band range is [in_kx_lo, in_kx_lo + in_kx_n)
  // (the frame's own band unless several modalities share one pass 1)
  const float2* band_in;
  int in_kx_lo, in_kx_n;
};

// ---- F1-F3: records, pixel boxes, pairs per particle; tile buckets -----------
// A one-digit counting sort on the tile key with fixed-size buckets: every pair
// (tile, particle) takes the next slot of its tile's bucket through an atomic
// cursor.  The counters must be zero on entry (k_bin_clear); they end as the
// tiles' true pair counts, which may exceed the bucket (the reader then falls
// back to an id-ordered scan for that tile, and scal[1] counts such tiles).  The
// order of ids inside a bucket is restored by the reader, which sorts it.
// A group of kBinGroup lanes shares one particle: its first lane writes the
// record, box and count, and the group deals the particle's tiles round robin,
// each lane issuing up to kFillBatch cursor increments before their results are
// used (a particle meets ~5 tiles on average, so most lanes wait on one
// increment instead of one lane on all of them).
constexpr int kBinGroup = 8;
constexpr int kFillBatch = 4;

__device__ __forceinline__ void bin_body(const FrameDev& F, int64_t gid) {
  const int64_t p = gid / kBinGroup;
  const int sub = (int)(gid - p * kBinGroup);
  if (p >= F.n) return;
  const float* soa = F.soa;
  const int64_t ld = F.ld;
  const float cx = soa[0 * ld + p], cy = soa[1 * ld + p], ang = soa[2 * ld + p];
  const float a = soa[3 * ld + p], b = soa[4 * ld + p], h = soa[5 * ld + p];
  const float dn = soa[6 * ld + p], shape = soa[7 * ld + p];
  int4 box;
  float R = 0.0f, habit = -1.0f;  // a polyhedral habit's bounding radius and index
  if (shape >= 1.5f) {
    const float kf = floorf(shape + 0.5f) - 2.0f;
    if (kf >= 0.0f && kf < (float)F.n_habits) {
      habit = kf;
      R = F.hab_info[(int)kf].y;
    }
  }
  const bool ok = pixel_box(cx, cy, a, b, shape, R, F.H, F.W, &box);
  int cnt = 0;
  if (ok) {
    const int tx0 = box.x / F.tile_w, tx1 = box.y / F.tile_w, ty0 = box.z / F.tile_h, ty1 = box.w / F.tile_h;
    cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
  }
  if (sub == 0) {
    PRec r;
#pragma unroll
    for (int k = 0; k < 32; ++k) r.f[k] = 0.0f;
    if (ok) {
      make_record(cx, cy, ang, a, b, h, dn, shape, R, habit, &r);
    } else {
      r.f[3] = -1.0f;
      box = make_int4(1, 0, 1, 0);
    }
    F.recs[p] = r;
    F.boxes[p] = box;
    if (F.absorb) {  // Beer-Lambert weight of the thickness (Eq. 4): row 8 holds dmu
      const float dmu = ok ? soa[8 * ld + p] : 0.0f;
      F.absr[p] = make_float2(dmu * h, dmu);
    }
    F.counts[p] = cnt;
  }
  if (ok) {
    const int tx0 = box.x / F.tile_w, tx1 = box.y / F.tile_w, ty0 = box.z / F.tile_h, ty1 = box.w / F.tile_h;
    const int nx = tx1 - tx0 + 1;
    const int cap = (int)F.cap;
    for (int e0 = sub; e0 < cnt; e0 += kBinGroup * kFillBatch) {
      int key[kFillBatch], pos[kFillBatch];
#pragma unroll
      for (int u = 0; u < kFillBatch; ++u) {
        const int e = e0 + u * kBinGroup;
        key[u] = e < cnt ? (ty0 + e / nx) * F.ntx + tx0 + e % nx : -1;
        pos[u] = key[u] >= 0 ? atomicAdd(&F.tile_count[key[u]], 1) : 0;
      }
#pragma unroll
      for (int u = 0; u < kFillBatch; ++u) {
        if (key[u] < 0) continue;
        if (pos[u] < cap) F.pids[(int64_t)key[u] * cap + pos[u]] = (int)p;
        else if (pos[u] == cap) atomicAdd(&F.scal[1], 1);
      }
    }
  }
}

// ---- inspection: exclusive prefix of the tile counts (one workgroup) -----------
// tile_first = prefix of the true counts; total pairs -> scal[3].  The counts
// pass through LDS in chunks of kScanChunk, read and written coalesced.
constexpr int kScanThreads = 1024;
constexpr int kScanChunk = 8192;

__device__ __forceinline__ void tile_scan_body(const FrameDev& F, long long* buf, long long* part) {
  const int t = threadIdx.x;
  const int nt = F.n_tiles;
  long long carry = 0;
  for (int c0 = 0; c0 < nt; c0 += kScanChunk) {
    const int cn = min(kScanChunk, nt - c0);
    for (int i = t; i < cn; i += kScanThreads) buf[i] = F.tile_count[c0 + i];
    __syncthreads();
    const int per = (cn + kScanThreads - 1) / kScanThreads;
    const int b0 = min(cn, t * per), b1 = min(cn, b0 + per);
    long long s = 0;
    for (int k = b0; k < b1; ++k) s += buf[k];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
      const long long v = t >= off ? part[t - off] : 0;
      __syncthreads();
      part[t] += v;
      __syncthreads();
    }
    long long run = carry + part[t] - s;
    for (int k = b0; k < b1; ++k) {
      const long long c = buf[k];
      buf[k] = run;
      run += c;
    }
    const long long chunk_total = part[kScanThreads - 1];
    __syncthreads();
    for (int i = t; i < cn; i += kScanThreads) F.tile_first[c0 + i] = (int)(buf[i] < INT_MAX ? buf[i] : INT_MAX);
    carry += chunk_total;
    __syncthreads();
  }
  if (t == 0) F.scal[3] = carry < INT_MAX ? (int)carry : INT_MAX;
}

// ---- F4: a tile's particle ids in ascending order, for one 64-lane wave -------
// The fill leaves each tile's ids in arbitrary order.  Up to 64 ids are sorted
// in registers (bitonic network over the lanes); up to kSegSort in LDS; a
// longer list is not materialised: the caller visits all particles in id order
// and keeps those whose box meets the tile (the same ids, the same order).
constexpr int kSegSort = kMaxBucket;

__device__ __forceinline__ int wave_sort64(int v, int lane) {
#pragma unroll
  for (int k = 2; k <= 64; k <<= 1)
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      const int o = __shfl_xor(v, j, 64);
      const bool keep_min = ((lane & j) == 0) == ((lane & k) == 0);
      v = keep_min ? min(v, o) : max(v, o);
    }
  return v;
}

// In-place ascending bitonic sort of seg[0, n2), n2 a power of two <= kSegSort,
// by the 64 lanes of a single-wave workgroup.
__device__ __forceinline__ void lds_sort(int* seg, int n2, int lane) {
  for (int k = 2; k <= n2; k <<= 1)
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int q = lane; q < n2 / 2; q += 64) {
        const int i = ((q & ~(j - 1)) << 1) | (q & (j - 1));  // q with a 0 inserted at bit log2(j)
        const int a = seg[i], b = seg[i + j];
        const bool asc = (i & k) == 0;
        if ((a > b) == asc) {
          seg[i] = b;
          seg[i + j] = a;
        }
      }
      __syncthreads();
    }
}

// ---- F5: rasterise one tile with one 64-lane wave ------------------------------
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

// A select the compiler keeps as v_cndmask (both operands already computed)
// rather than turning into a divergent branch.
__device__ __forceinline__ float sel(bool c, float x, float y) {
  return __builtin_unpredictable(c) ? x : y;
}

struct TileAcc {
  int pi[4], pj[4];          // canvas row and column of the lane's pixel in each slot
  float px[4], py[4];        // that pixel's centre, j + 1/2 and i + 1/2
  // every lane also holds the bounds of slot (lane & 3), so that the four
  // wave-uniform slot tests of a particle run as one vector instruction each
  float sx0, sx1, sy0, sy1;  // pixel-edge bounds of that slot (canvas pixels)
  float scx, scy, shx, shy;  // centre of its pixel centres, half extents
  float acc[4];
  float tacc[4];             // absorbance sums (absorbing frames)
  const float4* hab_enc;     // polyhedral habits of the frame
  const float4* hab_raw;
  const float4* hab_info;
  uint32_t topo_lo, topo_hi;
};

// Adds one particle to the four pixel slots a lane owns.  The slot tests (does
// the particle reach the slot; is every pixel centre of the slot deep inside a
// prism) are evaluated for the four slots at once, one slot per lane, and read
// back as wave-uniform bit masks: a slot the particle misses is skipped and a
// slot inside its footprint takes the full amplitude.  In any other slot every
// lane evaluates its pixel without branching for the common cases -- outside,
// inside, one edge (the half-plane box filter) for a prism; the centre sample for
// an ellipsoid -- and only marks the rare costly pixels: a prism pixel two edges
// reach (the clipped-polygon area) and an ellipsoid pixel within 2e-3 of the rim
// (FP64).  Those are evaluated after the four slots, each lane serving its own
// marks, so the costly code runs once per particle rather than once per slot.
// The offset of a pixel centre from the particle centre is exact in FP32 (both
// are multiples of the centre's ulp and the difference is small), so the rotated
// offsets u, v carry ~1e-6 px of rounding and depend on the pixel and the
// particle alone: the canvas is bitwise the same under every tiling.  Every
// pixel receives exactly one term per particle, in particle order.  ABS: the same
// coverage (prism) or centre thickness (ellipsoid) also adds dmu * height times it
// to the absorbance sums; ab = (dmu * height, dmu) of the particle.
template <bool ABS, bool HAB>
__device__ __forceinline__ void add_particle(const PRec& r, TileAcc& T, float2 ab) {
#pragma clang fp contract(off)
  const float kind = r.f[3];
  const float amp = r.f[2];
  unsigned marks = 0u;
  const float c = r.f[4], s = r.f[5];
  if (kind == 0.0f) {
    const float a = r.f[6], b = r.f[7];
    // half-plane box filter constants (as in halfplane_cover; (c, s) and (s, c) share them)
    const float hp_h = r.f[24], hp_l = r.f[25], hp_rp = r.f[26], hp_r2 = r.f[27];
    const float hd = hp_h + 1e-4f;  // pixel_half_extent(c, s)
    const bool a_ok = a >= hd, b_ok = b >= hd;  // the pixel cannot reach both edges of a pair
    unsigned hit_m, in_m;
    {  // slot (lane & 3): reached at all; every pixel centre deep inside both slabs
      const bool hit = !((r.f[21] <= T.sx0) | (r.f[20] >= T.sx1) | (r.f[23] <= T.sy0) | (r.f[22] >= T.sy1));
      const float sdx = T.scx - r.f[0], sdy = T.scy - r.f[1];
      const float uc = __builtin_fmaf(c, sdx, s * sdy), vc = __builtin_fmaf(c, sdy, -(s * sdx));
      const float ux = fabsf(uc) + fabsf(c) * T.shx + fabsf(s) * T.shy;
      const float vy = fabsf(vc) + fabsf(s) * T.shx + fabsf(c) * T.shy;
      const bool deep = (ux < a - hd) & (vy < b - hd);
      hit_m = (unsigned)__ballot(hit) & 15u;
      in_m = (unsigned)__ballot(hit & deep) & 15u;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!((hit_m >> q) & 1u)) continue;
      if ((in_m >> q) & 1u) {
        T.acc[q] += amp;
        if (ABS) T.tacc[q] += ab.x;
        continue;
      }
      // straight-line code: every case is a select.  A pixel two edges reach
      // takes 0 here and its clipped-polygon area below.
      const bool off_box = (T.px[q] >= r.f[29]) | (T.px[q] <= r.f[28]) | (T.py[q] >= r.f[31]) | (T.py[q] <= r.f[30]);
      const float dx = T.px[q] - r.f[0], dy = T.py[q] - r.f[1];
      const float u = __builtin_fmaf(c, dx, s * dy), v = __builtin_fmaf(c, dy, -(s * dx));
      const float du = fabsf(u) - a, dv = fabsf(v) - b;  // signed distances to the nearer edges
      const bool in_u = du < -hd, in_v = dv < -hd;
      const bool inside = in_u & in_v;
      const bool outside = off_box | (du > hd) | (dv > hd);
      const bool edge_u = in_v & a_ok;
      const bool edge = edge_u | (in_u & b_ok);
      // halfplane_cover(t, .) with t = -du (edge_u) or -dv; beyond the pixel's
      // half-extent e = 0, so the triangle term gives exactly 0 or 1
      const float t = edge_u ? -du : -dv;
      const float at = fabsf(t);
      const float e = fmaxf(hp_h - at, 0.0f);
      const float tri = e * e * hp_r2;
      const float lin = 0.5f + t * hp_rp;
      float cover = sel(t > 0.0f, 1.0f - tri, tri);
      cover = sel(at <= hp_l, lin, cover);
      cover = sel(edge, cover, 0.0f);
      cover = sel(inside, 1.0f, cover);
      cover = sel(outside, 0.0f, cover);
      T.acc[q] += amp * cover;
      if (ABS) T.tacc[q] += ab.x * cover;
      marks |= (unsigned)(!(outside | inside | edge)) << q;
    }
    while (marks) {
      const int q = __builtin_ctz(marks);
      marks &= marks - 1u;
      // one call site; selects keep the slot arrays in registers
      const int ii = q == 0 ? T.pi[0] : (q == 1 ? T.pi[1] : (q == 2 ? T.pi[2] : T.pi[3]));
      const int jj = q == 0 ? T.pj[0] : (q == 1 ? T.pj[1] : (q == 2 ? T.pj[2] : T.pj[3]));
      const float area = prism_clip_area(r, ii, jj);
      const float add = amp * area;
      if (q == 0) T.acc[0] += add;
      else if (q == 1) T.acc[1] += add;
      else if (q == 2) T.acc[2] += add;
      else T.acc[3] += add;
      if (ABS) {
        const float tadd = ab.x * area;
        if (q == 0) T.tacc[0] += tadd;
        else if (q == 1) T.tacc[1] += tadd;
        else if (q == 2) T.tacc[2] += tadd;
        else T.tacc[3] += tadd;
      }
    }
  } else if (kind == 1.0f) {
    // slot (lane & 3) meets the bounding box of the pixel centres the ellipse reaches
    const bool hit = !((T.sx1 - 0.5f - r.f[0] < -r.f[16]) | (T.sx0 + 0.5f - r.f[0] > r.f[16]) |
                       (T.sy1 - 0.5f - r.f[1] < -r.f[17]) | (T.sy0 + 0.5f - r.f[1] > r.f[17]));
    const unsigned hit_m = (unsigned)__ballot(hit) & 15u;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!((hit_m >> q) & 1u)) continue;
      const float dx = T.px[q] - r.f[0], dy = T.py[q] - r.f[1];
      const float u = __builtin_fmaf(c, dx, s * dy) * r.f[8], v = __builtin_fmaf(c, dy, -(s * dx)) * r.f[9];
      const float qv = u * u + v * v;
      // outside: 0; within 2e-3 of the rim: 0 here and the FP64 value below
      const bool rim = (qv > 0.998f) & (qv < 1.002f);
      // 1 - q >= 0.002 where the value is kept, so the hardware square root
      // (within 1 ulp, no denormal scaling needed) serves
      const float sq = sel(qv <= 0.998f, __builtin_amdgcn_sqrtf(fmaxf(1.0f - qv, 0.0f)), 0.0f);
      T.acc[q] += amp * sq;
      if (ABS) T.tacc[q] += ab.x * sq;
      marks |= (unsigned)rim << q;
    }
    while (marks) {
      const int q = __builtin_ctz(marks);
      marks &= marks - 1u;
      const int ii = q == 0 ? T.pi[0] : (q == 1 ? T.pi[1] : (q == 2 ? T.pi[2] : T.pi[3]));
      const int jj = q == 0 ? T.pj[0] : (q == 1 ? T.pj[1] : (q == 2 ? T.pj[2] : T.pj[3]));
      // h sqrt(1 - q) in FP64 with q recomputed in FP64, times dn (and dmu)
      const double qq = ellipsoid_rim_q(r, ii, jj);
      const double sq = qq < 1.0 ? sqrt(1.0 - qq) : 0.0;
      const float add = (float)((double)r.f[14] * (double)r.f[15] * sq);
      if (q == 0) T.acc[0] += add;
      else if (q == 1) T.acc[1] += add;
      else if (q == 2) T.acc[2] += add;
      else T.acc[3] += add;
      if (ABS) {
        const float tadd = (float)((double)ab.y * (double)r.f[15] * sq);
        if (q == 0) T.tacc[0] += tadd;
        else if (q == 1) T.tacc[1] += tadd;
        else if (q == 2) T.tacc[2] += tadd;
        else T.tacc[3] += tadd;
      }
    }
  } else if (HAB && kind == 2.0f) {
    // polyhedral habit: chord of the vertical ray through the pixel centre (Eq. 1),
    // times the height, plus the micro-topography where it is positive
    const bool hit = !((T.sx1 - 0.5f - r.f[0] < -r.f[16]) | (T.sx0 + 0.5f - r.f[0] > r.f[16]) |
                       (T.sy1 - 0.5f - r.f[1] < -r.f[17]) | (T.sy0 + 0.5f - r.f[1] > r.f[17]));
    const unsigned hit_m = (unsigned)__ballot(hit) & 15u;
    const int k = (int)r.f[18];
    const float4 info = T.hab_info[k];
    const float4* __restrict__ enc = T.hab_enc + k * kMaxFaces;
    const int nf = (int)info.x;
    const float h = r.f[15], dn = r.f[14], tamp = info.z, inv_cell = 1.0f / info.w;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (!((hit_m >> q) & 1u)) continue;
      const float dx = T.px[q] - r.f[0], dy = T.py[q] - r.f[1];
      const float U = __builtin_fmaf(c, dx, s * dy) * r.f[8], V = __builtin_fmaf(c, dy, -(s * dx)) * r.f[9];
      float near;
      float t = h * habit_chord(enc, nf, U, V, &near);
      if (tamp > 0.0f && t > 0.0f)
        t = fmaxf(t + tamp * value_noise(T.px[q], T.py[q], inv_cell, (uint32_t)k, T.topo_lo, T.topo_hi), 0.0f);
      const bool costly = near < 1e-4f;  // next to a vertical face: FP64 below
      T.acc[q] += sel(costly, 0.0f, dn * t);
      if (ABS) T.tacc[q] += sel(costly, 0.0f, ab.y * t);
      marks |= (unsigned)costly << q;
    }
    while (marks) {
      const int q = __builtin_ctz(marks);
      marks &= marks - 1u;
      const int ii = q == 0 ? T.pi[0] : (q == 1 ? T.pi[1] : (q == 2 ? T.pi[2] : T.pi[3]));
      const int jj = q == 0 ? T.pj[0] : (q == 1 ? T.pj[1] : (q == 2 ? T.pj[2] : T.pj[3]));
      double t = (double)h * habit_chord64(r, T.hab_raw + k * kMaxFaces, nf, ii, jj);
      if (tamp > 0.0f && t > 0.0)
        t = fmax(t + (double)tamp * (double)value_noise((float)jj + 0.5f, (float)ii + 0.5f, inv_cell, (uint32_t)k,
                                                        T.topo_lo, T.topo_hi), 0.0);
      const float add = (float)((double)dn * t);
      if (q == 0) T.acc[0] += add;
      else if (q == 1) T.acc[1] += add;
      else if (q == 2) T.acc[2] += add;
      else T.acc[3] += add;
      if (ABS) {
        const float tadd = (float)((double)ab.y * t);
        if (q == 0) T.tacc[0] += tadd;
        else if (q == 1) T.tacc[1] += tadd;
        else if (q == 2) T.tacc[2] += tadd;
        else T.tacc[3] += tadd;
      }
    }
  }
}

// Lane `lane` of the wave owns pixels lane, lane+64, lane+128, lane+192 of the
// tile.  The particle loop, the record load (scalar cache) and the kind dispatch
// run once per (tile, particle); ids are fetched 64 at a time and broadcast.
// Particles are visited in ascending id: the tile's bucket is sorted on the fly
// (wave_sort64 / lds_sort); a tile whose bucket overflowed is served by a scan of
// all particles in id order that keeps those whose box meets the tile.  All three visit the same
// particles in the same order, so the sums are identical.  `seg`: kSegSort ints
// of LDS; the workgroup is this single wave.
template <bool ABS>
__device__ __forceinline__ float2 absorb_weights(const FrameDev& F, int64_t id) {
  return ABS ? F.absr[id] : make_float2(0.0f, 0.0f);
}

template <bool ABS, bool HAB>
__device__ __forceinline__ void raster_ids(const FrameDev& F, TileAcc& T, int mine, int m) {
#pragma clang fp contract(off)
  const PRec* __restrict__ recs = F.recs;
  PRec nxt = recs[__builtin_amdgcn_readlane(mine, 0)];
  for (int k = 0; k < m; ++k) {
    const PRec cur = nxt;
    const float2 ab = absorb_weights<ABS>(F, __builtin_amdgcn_readlane(mine, k));
    if (k + 1 < m) nxt = recs[__builtin_amdgcn_readlane(mine, k + 1)];
    add_particle<ABS, HAB>(cur, T, ab);
  }
}

template <bool ABS, bool HAB>
__device__ __forceinline__ void raster_tile(const FrameDev& F, int tile, int lane, int* seg) {
#pragma clang fp contract(off)
  const int tile_w = F.tile_w, tile_h = F.tile_h;
  const int ty = tile / F.ntx, tx = tile - ty * F.ntx;
  TileAcc T;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = lane + 64 * k, li = q / tile_w, lj = q - li * tile_w;
    T.pi[k] = ty * tile_h + li;
    T.pj[k] = tx * tile_w + lj;
    T.px[k] = (float)T.pj[k] + 0.5f;
    T.py[k] = (float)T.pi[k] + 0.5f;
    T.acc[k] = 0.0f;
    T.tacc[k] = 0.0f;
  }
  T.hab_enc = F.hab_enc;
  T.hab_raw = F.hab_raw;
  T.hab_info = F.hab_info;
  T.topo_lo = F.topo_lo;
  T.topo_hi = F.topo_hi;
  {
    const SubRect R = slot_rect(64 * (lane & 3), tile_w, tx, ty, tile_h);
    T.sx0 = R.x0;
    T.sx1 = R.x1;
    T.sy0 = R.y0;
    T.sy1 = R.y1;
    T.scx = 0.5f * (R.x0 + R.x1);
    T.scy = 0.5f * (R.y0 + R.y1);
    T.shx = 0.5f * (R.x1 - R.x0 - 1.0f);
    T.shy = 0.5f * (R.y1 - R.y0 - 1.0f);
  }
  const int cnt = F.tile_count[tile];
  const bool overflow = cnt > (int)F.cap;     // the bucket could not hold the tile's ids
  const int* __restrict__ pids = F.pids + (int64_t)tile * F.cap;
  const int start = 0;
  if (!overflow && cnt <= 64) {
    if (cnt > 0) {
      const int mine = wave_sort64(lane < cnt ? pids[start + lane] : INT_MAX, lane);
      raster_ids<ABS, HAB>(F, T, mine, cnt);
    }
  } else if (!overflow && cnt <= kSegSort) {
    int n2 = 128;
    while (n2 < cnt) n2 <<= 1;
    for (int i = lane; i < n2; i += 64) seg[i] = i < cnt ? pids[start + i] : INT_MAX;
    __syncthreads();
    lds_sort(seg, n2, lane);
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      const int m = min(64, cnt - c0);
      raster_ids<ABS, HAB>(F, T, lane < m ? seg[c0 + lane] : 0, m);
    }
  } else {
    const int x0 = tx * tile_w, x1 = x0 + tile_w - 1, y0 = ty * tile_h, y1 = y0 + tile_h - 1;
    for (int64_t p = 0; p < F.n; ++p) {
      const int4 b = F.boxes[p];
      if (b.x > b.y || b.x > x1 || b.y < x0 || b.z > y1 || b.w < y0) continue;
      add_particle<ABS, HAB>(F.recs[p], T, absorb_weights<ABS>(F, p));
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    F.opd[(int64_t)T.pi[q] * F.W + T.pj[q]] = T.acc[q];
    if (ABS) F.tau[(int64_t)T.pi[q] * F.W + T.pj[q]] = T.tacc[q];
  }
}

// ---- F6: pass 1, rows --------------------------------------------------------
// Workgroup g transforms rows [g RPB, (g + 1) RPB); the band keeps its row blocks
// of RB >= RPB rows, so a workgroup fills RPB of the RB entries of each column.
template <int LOGW, int MAXR>
__device__ __forceinline__ void pass1_body(const FrameDev& F, int g, const float2* __restrict__ tw, char* lds) {
#pragma clang fp contract(off)
  constexpr int W = 1 << LOGW, RB = rows_per_block(W), RPB = rows_per_fft_block(W);
  float2* buf = reinterpret_cast<float2*>(lds);
  const int t = threadIdx.x;
  const float* src = F.opd + (size_t)g * RPB * W;
  const float pk = F.phase_k;
  // every load of the row block is issued before the first is used, so the
  // workgroup waits on memory once rather than once per point it handles
  constexpr int PER = RPB * W / kThreads;
  static_assert(RPB * W % kThreads == 0, "row block not a multiple of the workgroup");
  float ph[PER];
#pragma unroll
  for (int u = 0; u < PER; ++u) ph[u] = src[t + u * kThreads];
  if (F.absorb) {  // U = exp(-tau) exp(i phi): the Beer-Lambert amplitude of Eq. 4
    const float* ta = F.tau + (size_t)g * RPB * W;
    float tv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) tv[u] = ta[t + u * kThreads];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      float s, c;
      sincosf(pk * ph[u], &s, &c);
      const float am = expf(-tv[u]);
      buf[t + u * kThreads] = make_float2(am * c, am * s);
    }
  } else {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      float s, c;
      sincosf(pk * ph[u], &s, &c);
      buf[t + u * kThreads] = make_float2(c, s);
    }
  }
  __syncthreads();
  Stages<W, RPB, -1, 1, LOGW, MAXR>::run(buf, tw);
  const int kx_lo = F.o.kx_lo, kx_n = F.o.kx_n;
  const int row0 = g * RPB, blk = row0 / RB, r0 = row0 % RB;
  float2* dst = F.band + (size_t)blk * kx_n * RB + r0;
  for (int idx = t; idx < kx_n * RPB; idx += kThreads) {
    const int b = idx / RPB, r = idx - b * RPB;
    dst[(size_t)b * RB + r] = buf[r * W + ((kx_lo + b) & (W - 1))];
  }
  __syncthreads();
}

// ---- F7: pass 2, one in-band column ------------------------------------------
template <int LOGH, int MAXR>
__device__ __forceinline__ void pass2_body(const FrameDev& F, int b, const float2* __restrict__ tw, char* lds) {
#pragma clang fp contract(off)
  constexpr int H = 1 << LOGH;
  float2* buf = reinterpret_cast<float2*>(lds);
  double* red = reinterpret_cast<double*>(lds + fft_lds_f2(H) * sizeof(float2));
  int* chord = reinterpret_cast<int*>(lds + fft_lds_f2(H) * sizeof(float2) + kThreads * sizeof(double));
  const OpticsArgs& o = F.o;
  const int t = threadIdx.x, kx = o.kx_lo + b;
  const int RB = o.rb;
  float2* band = F.band;
  const float2* src = F.band_in;
  const int bi = kx - F.in_kx_lo, in_n = F.in_kx_n;
  {  // the column's loads all in flight before the first is used
    constexpr int PER = (H + kThreads - 1) / kThreads;
    float2 v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = t + u * kThreads;
      if (H % kThreads == 0 || i < H) v[u] = src[((size_t)(i / RB) * in_n + bi) * RB + (i % RB)];
    }
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      const int i = t + u * kThreads;
      if (H % kThreads == 0 || i < H) buf[i] = v[u];
    }
  }
  if (t == 0) band_chord(o, kx, &chord[0], &chord[1]);
  __syncthreads();
  Stages<H, 1, -1, 1, LOGH, MAXR>::run(buf, tw);
  const float dz = F.globals[0], shear = F.globals[1], bias = F.globals[2];
  const int lo = chord[0], hi = chord[1];
  double part = 0.0;
  for (int m = t; m < H; m += kThreads) {
    const int ky = m < H / 2 ? m : m - H;
    float2 g = make_float2(0.0f, 0.0f);
    if (ky >= lo && ky <= hi) {
      g = cmul(buf[m], transfer(o, kx, ky, dz, shear, bias));
      part += (double)g.x * g.x + (double)g.y * g.y;
    }
    buf[m] = g;
  }
  const double colsum = block_sum(part, red);  // its barriers also order buf for the stages
  if (t == 0) F.colsum[b] = colsum;
  Stages<H, 1, 1, 1, LOGH, MAXR>::run(buf, tw);
  for (int i = t; i < H; i += kThreads) band[((size_t)(i / RB) * o.kx_n + b) * RB + (i % RB)] = buf[i];
  __syncthreads();
}

// ---- F8: pass 3, rows: inverse FFT from the band, |E|^2, shot noise ------------
// With noise, every workgroup forms the photon scale s = photons / mean(I) from
// the per-column Parseval sums of pass 2 (the same fixed summation order in every
// workgroup, so all agree bit for bit) and samples its rows' counts in place:
// I <- Poisson(s I) / s.  Pixels 2m, 2m+1 share the Philox block (m, frame, 0, 0).
//
// Sampling is split so that the costly branch runs on compacted work: every lane
// first draws its pixels' shared blocks and applies the PTRS squeeze (or the
// inversion for means below 10); pixels the squeeze does not settle go, with
// their two words, to a per-wave queue in LDS, which the wave then drains with
// all lanes busy (full PTRS attempt, then own blocks).  Each pixel's arithmetic
// is exactly that of poisson().
constexpr int kNoiseChunk = 4;                                   // pairs per lane per round
constexpr int kNoiseQueueBytes = kThreads * 2 * kNoiseChunk * 16;  // uint4 entries, 32 KB

__host__ __device__ constexpr int pass3_buf_bytes(int W) {
  return fft_lds_f2(rows_per_fft_block(W) * W) * 8 > kNoiseQueueBytes ? fft_lds_f2(rows_per_fft_block(W) * W) * 8
                                                                       : kNoiseQueueBytes;
}

// Orders LDS accesses among the lanes of one wave: enough for a wave-private
// region, where a workgroup barrier would also wait for the other waves.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Inclusive prefix sum over the 64 lanes of a wave.
__device__ __forceinline__ int wave_incl_scan(int v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int u = __shfl_up(v, d, 64);
    if (lane >= d) v += u;
  }
  return v;
}

template <int NP>
__device__ __forceinline__ void noise_rows(const FrameDev& F, float scale, int64_t pix0, const float* Ipix,
                                           float* dst, char* lds) {
#pragma clang fp contract(off)
  constexpr int PP = (NP + kThreads - 1) / kThreads;  // pairs per thread
  constexpr int CH = PP < kNoiseChunk ? PP : kNoiseChunk;
  const OpticsArgs& o = F.o;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  uint4* queue = reinterpret_cast<uint4*>(lds) + wave * (64 * 2 * CH);
  const float inv_scale = 1.0f / scale;  // counts / s as one multiply (within two ulps of the quotient)
  float2* out = reinterpret_cast<float2*>(dst);
  for (int k0 = 0; k0 < PP; k0 += CH) {
    float res[2 * CH];
    uint4 ent[2 * CH];
    unsigned pend = 0u;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int ml = t + kThreads * (k0 + c);
      res[2 * c] = 0.0f;
      res[2 * c + 1] = 0.0f;
      if (ml >= NP) continue;
      const int64_t p = pix0 + 2 * ml;
      const uint32_t m = (uint32_t)(p >> 1);
      const uint4 r = philox4x32_10(make_uint4(m, o.frame, 0u, 0u), o.seed_lo, o.seed_hi);
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        const float mu = scale * Ipix[2 * (k0 + c) + x];
        const uint32_t w0 = x ? r.z : r.x, w1 = x ? r.w : r.y;
        if (!(mu > 0.0f)) {
          res[2 * c + x] = 0.0f;
        } else if (mu < 10.0f) {
          res[2 * c + x] = (float)poisson_small(mu, w0);
        } else {
          const PtrsConst pc = ptrs_const(mu);
          float U, V, us, kf;
          if (ptrs_quick(w0, w1, mu, pc.a, pc.b, pc.vr, &U, &V, &us, &kf)) {
            res[2 * c + x] = (float)(int)kf;
          } else {
            pend |= 1u << (2 * c + x);
            ent[2 * c + x] = make_uint4((uint32_t)(p + x), __float_as_uint(mu), w0, w1);
          }
        }
      }
    }
    // compact the unsettled pixels into the wave's queue
    const int cnt = __popc(pend);
    const int incl = wave_incl_scan(cnt, lane);
    const int total = __shfl(incl, 63, 64);
    int pos = incl - cnt;
#pragma unroll
    for (int e = 0; e < 2 * CH; ++e)
      if (pend & (1u << e)) queue[pos++] = ent[e];
    wave_sync();
    for (int q = lane; q < total; q += 64) {
      const uint4 en = queue[q];
      const int k = poisson_large(__uint_as_float(en.y), en.z, en.w, en.x, o.frame, o.seed_lo, o.seed_hi);
      queue[q].y = (uint32_t)k;
    }
    wave_sync();
    pos = incl - cnt;
#pragma unroll
    for (int e = 0; e < 2 * CH; ++e)
      if (pend & (1u << e)) res[e] = (float)(int)queue[pos++].y;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int ml = t + kThreads * (k0 + c);
      if (ml >= NP) continue;
      float a = res[2 * c], b = res[2 * c + 1];
      if (o.read_sigma > 0.0f) {  // Gaussian read noise: Box-Muller on the pair's own block
        const uint32_t m = (uint32_t)((pix0 + 2 * ml) >> 1);
        const uint4 w = philox4x32_10(make_uint4(m, o.frame, 0u, 2u), o.seed_lo, o.seed_hi);
        const float r = sqrtf(-2.0f * logf(u01(w.x)));
        float sn, cs;
        sincosf(6.283185307179586f * u01(w.y), &sn, &cs);
        a = a + o.read_sigma * (r * cs);
        b = b + o.read_sigma * (r * sn);
      }
      out[ml] = make_float2(a * inv_scale, b * inv_scale);
    }
    wave_sync();  // the wave's queue is reused by the next round
  }
}

template <int LOGW, int MAXR>
__device__ __forceinline__ void pass3_body(const FrameDev& F, int g, const float2* __restrict__ tw, char* lds) {
#pragma clang fp contract(off)
  constexpr int W = 1 << LOGW, RB = rows_per_block(W), RPB = rows_per_fft_block(W), NP = RPB * W / 2;
  constexpr int PP = (NP + kThreads - 1) / kThreads;
  float2* buf = reinterpret_cast<float2*>(lds);
  double* red = reinterpret_cast<double*>(lds + pass3_buf_bytes(W));
  const OpticsArgs& o = F.o;
  const int t = threadIdx.x;
  for (int idx = t; idx < RPB * W; idx += kThreads) buf[idx] = make_float2(0.0f, 0.0f);
  __syncthreads();
  const int row0 = g * RPB, blk = row0 / RB, r0 = row0 % RB;
  const float2* src = F.band + (size_t)blk * o.kx_n * RB + r0;
  constexpr int LB = 4;  // band loads in flight per thread
  const int nb = o.kx_n * RPB;
  for (int i0 = t; i0 < nb; i0 += LB * kThreads) {
    float2 v[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int idx = i0 + u * kThreads, b = idx / RPB, r = idx - b * RPB;
      if (idx < nb) v[u] = src[(size_t)b * RB + r];
    }
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int idx = i0 + u * kThreads, b = idx / RPB, r = idx - b * RPB;
      if (idx < nb) buf[r * W + ((o.kx_lo + b) & (W - 1))] = v[u];
    }
  }
  const bool noise = o.photons > 0.0f;
  __syncthreads();
  float scale = 0.0f;
  if (noise) {  // o.photons is uniform over the workgroup, so the barriers inside are too
    double s = 0.0;
    for (int b = t; b < o.colsum_n; b += kThreads) s += F.colsum[b];
    const double hw = (double)o.H * (double)W;
    const double mean = block_sum(s, red) / (hw * hw);
    scale = mean > 0.0 ? (float)((double)o.photons / mean) : 0.0f;
  }
  Stages<W, RPB, 1, 1, LOGW, MAXR>::run(buf, tw);
  const float inv = o.inv_hw;
  float* dst = F.intensity + (size_t)row0 * W;
  // coherent modes: I = |E|^2; incoherent DIC: the band holds the spectrum of I
  // itself (real up to rounding), so I = Re
  const bool real_part = o.mode == OSOG_DIC_INCOHERENT;
  if (!(scale > 0.0f)) {
    for (int idx = t; idx < RPB * W; idx += kThreads) {
      const float2 e = buf[idx];
      const float er = e.x * inv, ei = e.y * inv;
      dst[idx] = real_part ? er : er * er + ei * ei;
    }
    __syncthreads();
    return;
  }
  // intensities of this thread's pixel pairs (ml = t + 256 k), then the LDS is free
  float Ipix[2 * PP];
#pragma unroll
  for (int k = 0; k < PP; ++k) {
    const int ml = t + kThreads * k;
    // the pair's two fields in one 16-byte read (consecutive lanes, consecutive banks)
    const float4 e2 = ml < NP ? reinterpret_cast<const float4*>(buf)[ml] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      const float er = (x ? e2.z : e2.x) * inv, ei = (x ? e2.w : e2.y) * inv;
      Ipix[2 * k + x] = ml < NP ? (real_part ? fmaxf(er, 0.0f) : er * er + ei * ei) : 0.0f;  // a Poisson mean is >= 0
    }
  }
  __syncthreads();
  noise_rows<NP>(F, scale, (int64_t)row0 * W, Ipix, dst, lds);
}

}  // namespace osog

namespace osog {

// Host: device descriptor of a planned frame on its carved workspace.  The
// caller sets soa / globals / opd / intensity.
inline FrameDev make_dev(const FramePlan& p, const FrameBufs& b) {
  FrameDev F{};
  F.H = p.H; F.W = p.W; F.logH = p.logH; F.logW = p.logW;
  F.tile_h = p.tile_h; F.tile_w = p.tile_w; F.ntx = p.ntx; F.n_tiles = p.n_tiles;
  F.n = p.n; F.ld = p.ld; F.cap = p.cap;
  F.o = optics_args(p);
  F.phase_k = p.phase_k;
  F.recs = b.recs; F.boxes = b.boxes; F.counts = b.counts; F.scal = b.scal;
  F.tile_count = b.tile_count; F.tile_first = b.tile_first;
  F.pids = b.pids;
  F.band = b.band; F.colsum = b.colsum;
  F.band_in = b.band; F.in_kx_lo = p.kx_lo; F.in_kx_n = p.kx_n;
  F.fft_radix = p.fft_radix;
  F.opd = b.opd;
  F.tau = b.tau;
  F.absr = b.absr;
  F.absorb = p.absorb;
  F.hab_enc = p.hab_enc;
  F.hab_raw = p.hab_raw;
  F.hab_info = p.hab_info;
  F.n_habits = p.n_habits;
  F.topo_lo = p.topo_lo;
  F.topo_hi = p.topo_hi;
  return F;
}

}  // namespace osog
