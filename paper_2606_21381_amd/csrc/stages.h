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
  int64_t n, ld;
  int64_t pair_cap;                // entries of the pair list
  OpticsArgs o;
  float phase_k;
  float inv_lambda;                // 1 / lambda [turns/um]
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
  int* scal;                       // [1] tiles rasterised by the id-ordered scan, [3] total pairs
  int* tile_count;                 // pairs per tile (histogram)
  int* tile_start;                 // n_tiles + 1: first pair of each tile's segment
  int* cursor;                     // next free entry of each segment (emit)
  int* items;                      // (tile << 4 | slice) of every plane in use
  int* tile_plane;                 // first plane of a sliced tile (-1: none left)
  int* tile_done;                  // slices of each tile finished (cleared per frame)
  unsigned long long* planes;      // plane_cap planes of tile sums
  int plane_cap;
  int* pids;                       // the pair list: particle ids grouped by tile
  float2* band;
  double* colsum;
  // pass 2 reads its columns from band_in, whose in-band range is [in_kx_lo, in_kx_lo + in_kx_n)
  // (the frame's own band unless several modalities share one pass 1)
  const float2* band_in;
  int in_kx_lo, in_kx_n;
};

// ---- F1: records, pixel boxes, pairs per particle, tile histogram ----------------
// A group of kBinGroup lanes shares one particle: its first lane writes the
// record, box and pair count, and the group deals the particle's tiles round
// robin, each lane adding one to the count of its tiles (integer atomics: the
// histogram does not depend on their order).  The histogram must be zero on
// entry (k_bin_clear).
constexpr int kBinGroup = 8;

__device__ __forceinline__ void bin_body(const FrameDev& F, int64_t gid) {
  const int64_t p = gid / kBinGroup;
  const int sub = (int)(gid - p * kBinGroup);
  if (p >= F.n) return;
  const float* soa = F.soa;
  const int64_t ld = F.ld;
  const float cx = soa[0 * ld + p], cy = soa[1 * ld + p];
  const float a = soa[3 * ld + p], b = soa[4 * ld + p], shape = soa[7 * ld + p];
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
  int tx0 = 0, ty0 = 0, nx = 0, cnt = 0;
  if (ok) {
    tx0 = box.x / F.tile_w;
    ty0 = box.z / F.tile_h;
    nx = box.y / F.tile_w - tx0 + 1;
    cnt = nx * (box.w / F.tile_h - ty0 + 1);
  }
  for (int e = sub; e < cnt; e += kBinGroup) atomicAdd(&F.tile_count[(ty0 + e / nx) * F.ntx + tx0 + e % nx], 1);
  if (sub == 0) {
    const float ang = soa[2 * ld + p], h = soa[5 * ld + p], dn = soa[6 * ld + p];
    PRec r;
    if (ok) {
      make_record(cx, cy, ang, a, b, h, dn, shape, R, habit, &r);
    } else {
#pragma unroll
      for (int k = 0; k < 32; ++k) r.f[k] = 0.0f;
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
}

// ---- F2: exclusive prefix of the tile histogram (one workgroup) -----------------
// tile_start[t] = pairs of tiles 0..t-1, tile_start[n_tiles] = all pairs (also
// scal[3]), and the emit cursors start at tile_start.  The counts pass through
// registers in chunks of kScanChunk, read and written coalesced; each thread sums
// kScanPer consecutive counts, the threads' sums are scanned across the wave with
// shuffles and across the waves in LDS.  Integer sums: the result is exact in any
// order.
// The same pass plans the slices of crowded tiles: a stored segment of more than
// kSlicePairs particles is split into S = ceil(count / kSlicePairs) slices (at
// most kMaxSlices), each rasterised by its own workgroup into its own plane of
// tile sums; tiles take consecutive planes in tile order while plane_cap lasts
// (tile_plane[t], -1 once they run out), and items lists (tile << 4 | slice) for
// every plane in use, scal[2] of them.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 16;                         // counts per thread and chunk
constexpr int kScanChunk = kScanThreads * kScanPer;  // 16384 tiles per pass
constexpr int kSlicePairs = 48;  // particles per slice of a crowded tile
constexpr int kMaxSlices = 16;

__device__ __forceinline__ long long wave_incl_scan(long long v, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const long long u = __shfl_up(v, o, 64);
    if (lane >= o) v += u;
  }
  return v;
}

// Slices of a stored segment of cnt particles.
__host__ __device__ __forceinline__ int tile_slices(int cnt) {
  return cnt > kSlicePairs ? min(kMaxSlices, (cnt + kSlicePairs - 1) / kSlicePairs) : 1;
}

// Exclusive prefix of s over the workgroup's threads (in thread order) plus the
// workgroup total.  wsum: 2 * kScanThreads / 64 + 1 long longs of LDS.
__device__ __forceinline__ long long block_excl_scan(long long s, long long* wsum, long long* total) {
  constexpr int NW = kScanThreads / 64;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const long long incl = wave_incl_scan(s, lane);
  if (lane == 63) wsum[wv] = incl;
  __syncthreads();
  if (wv == 0) {
    const long long w = lane < NW ? wsum[lane] : 0;
    const long long wi = wave_incl_scan(w, lane);
    if (lane < NW) wsum[NW + lane] = wi - w;  // exclusive per wave
    if (lane == NW - 1) wsum[2 * NW] = wi;    // workgroup total
  }
  __syncthreads();
  const long long ex = wsum[NW + wv] + incl - s;
  *total = wsum[2 * NW];
  __syncthreads();  // wsum is reused by the next scan
  return ex;
}

// Each thread holds kScanPer consecutive counts in registers (read as int4), so a
// chunk costs one round trip to memory.
__device__ __forceinline__ void tile_scan_body(const FrameDev& F, long long* wsum) {
  const int t = threadIdx.x;
  const int nt = F.n_tiles;
  long long carry = 0, ecarry = 0;
  for (int c0 = 0; c0 < nt; c0 += kScanChunk) {
    const int i0 = c0 + t * kScanPer;
    int loc[kScanPer];
    if (i0 + kScanPer <= nt) {  // n_tiles and c0 are multiples of 16 except on tiny canvases
      const int4* src = reinterpret_cast<const int4*>(F.tile_count + i0);
#pragma unroll
      for (int q = 0; q < kScanPer / 4; ++q) {
        const int4 v = src[q];
        loc[4 * q] = v.x; loc[4 * q + 1] = v.y; loc[4 * q + 2] = v.z; loc[4 * q + 3] = v.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) loc[k] = i0 + k < nt ? F.tile_count[i0 + k] : 0;
    }
    long long s = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) s += loc[k];
    long long tot;
    long long run = carry + block_excl_scan(s, wsum, &tot);
    carry += tot;
    int out[kScanPer], planes[kScanPer];
    int es = 0;
#pragma unroll
    for (int k = 0; k < kScanPer; ++k) {
      out[k] = run < INT_MAX ? (int)run : INT_MAX;
      run += loc[k];
      // only stored segments are sliced
      const int S = (i0 + k < nt && run <= (long long)F.pair_cap) ? tile_slices(loc[k]) : 1;
      planes[k] = S > 1 ? S : 0;
      es += planes[k];
    }
    if (i0 + kScanPer <= nt) {
      int4* d0 = reinterpret_cast<int4*>(F.tile_start + i0);  // tile_start is 16-byte aligned
      int4* d1 = reinterpret_cast<int4*>(F.cursor + i0);
#pragma unroll
      for (int q = 0; q < kScanPer / 4; ++q) {
        const int4 v = make_int4(out[4 * q], out[4 * q + 1], out[4 * q + 2], out[4 * q + 3]);
        d0[q] = v;
        d1[q] = v;
      }
    } else {
#pragma unroll
      for (int k = 0; k < kScanPer; ++k)
        if (i0 + k < nt) {
          F.tile_start[i0 + k] = out[k];
          F.cursor[i0 + k] = out[k];
        }
    }
    if (__syncthreads_or(es)) {  // some tile of the chunk is sliced: give it planes
      long long etot;
      int pp = (int)min(ecarry + block_excl_scan(es, wsum, &etot), (long long)INT_MAX);
      ecarry += etot;
#pragma unroll
      for (int k = 0; k < kScanPer; ++k) {
        if (planes[k] == 0) continue;
        if (pp + planes[k] <= F.plane_cap) {
          F.tile_plane[i0 + k] = pp;
          for (int j = 0; j < planes[k]; ++j) F.items[pp + j] = ((i0 + k) << 4) | j;
          atomicMax(&F.scal[2], pp + planes[k]);
        } else {
          F.tile_plane[i0 + k] = -1;
        }
        pp += planes[k];
      }
    }
  }
  if (t == 0) {
    const int tot = carry < INT_MAX ? (int)carry : INT_MAX;
    F.tile_start[nt] = tot;
    F.scal[3] = tot;
  }
}
// ---- F3: emit each pair into its tile's segment -----------------------------------
// A group of kBinGroup lanes shares one particle and deals its tiles round robin;
// every pair takes the next entry of its tile's segment through the tile's
// cursor.  The order inside a segment depends on the atomics and does not matter
// to the raster, whose sums are exact integers; only the inspection copy
// (k_sort_segments) is put in ascending id.  Pairs past the list's capacity are not
// stored (their tiles are rasterised by the scan over all particles instead).
constexpr int kFillBatch = 4;

__device__ __forceinline__ void emit_body(const FrameDev& F, int64_t gid) {
  const int64_t p = gid / kBinGroup;
  const int sub = (int)(gid - p * kBinGroup);
  if (p >= F.n) return;
  const int4 box = F.boxes[p];
  if (box.x > box.y) return;
  const int tx0 = box.x / F.tile_w, tx1 = box.y / F.tile_w, ty0 = box.z / F.tile_h, ty1 = box.w / F.tile_h;
  const int nx = tx1 - tx0 + 1, cnt = nx * (ty1 - ty0 + 1);
  for (int e0 = sub; e0 < cnt; e0 += kBinGroup * kFillBatch) {
    int pos[kFillBatch];
#pragma unroll
    for (int u = 0; u < kFillBatch; ++u) {
      const int e = e0 + u * kBinGroup;
      const int key = e < cnt ? (ty0 + e / nx) * F.ntx + tx0 + e % nx : -1;
      pos[u] = key >= 0 ? atomicAdd(&F.cursor[key], 1) : -1;
    }
#pragma unroll
    for (int u = 0; u < kFillBatch; ++u)
      if (pos[u] >= 0 && pos[u] < F.pair_cap) F.pids[pos[u]] = (int)p;
  }
}

// ---- F4 (inspection): a segment's particle ids in ascending order, one wave ------
// Up to 64 ids are sorted in registers (bitonic network over the lanes), up to
// kSegSort in LDS and then held in registers, kSegRegs per lane, so that the LDS
// used for the sort is free again while the ids are visited.  A longer segment,
// or one cut short by the list's capacity, is not sorted: the reader visits all
// particles in id order and keeps those whose box meets the tile (the same ids in
// the same order).
constexpr int kSegSort = 1024;
constexpr int kSegRegs = kSegSort / 64;

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

// Does particle p's box meet the tile [x0, x1] x [y0, y1]?
__device__ __forceinline__ bool box_meets(const FrameDev& F, int64_t p, int x0, int x1, int y0, int y1) {
  const int4 b = F.boxes[p];
  return !(b.x > b.y || b.x > x1 || b.y < x0 || b.z > y1 || b.w < y0);
}

// A tile's sorted segment as the lanes hold it: id c * 64 + lane in v[c].
struct TileIds {
  int v[kSegRegs];
  int cnt;    // ids in the segment
  bool scan;  // not stored or too long: read by the id-ordered scan instead
};

// Reads and sorts tile `tile`'s segment.  `seg`: seg_cap ints of LDS (a power of
// two, 128 <= seg_cap <= kSegSort), free again on return (the workgroup is one wave).
__device__ __forceinline__ TileIds tile_ids(const FrameDev& F, int tile, int lane, int* seg, int seg_cap) {
  TileIds T;
  const int start = F.tile_start[tile], end = F.tile_start[tile + 1];
  T.cnt = end - start;
  T.scan = !(end <= F.pair_cap && T.cnt <= seg_cap);
#pragma unroll
  for (int c = 0; c < kSegRegs; ++c) T.v[c] = 0;
  if (T.scan || T.cnt == 0) return T;
  const int* __restrict__ pids = F.pids + start;
  if (T.cnt <= 64) {
    T.v[0] = wave_sort64(lane < T.cnt ? pids[lane] : INT_MAX, lane);
  } else {
    int n2 = 128;
    while (n2 < T.cnt) n2 <<= 1;
    for (int i = lane; i < n2; i += 64) seg[i] = i < T.cnt ? pids[i] : INT_MAX;
    __syncthreads();
    lds_sort(seg, n2, lane);
#pragma unroll
    for (int c = 0; c < kSegRegs; ++c)
      if (c * 64 < T.cnt) T.v[c] = seg[c * 64 + lane];  // c * 64 + lane < n2
    __syncthreads();
  }
  return T;
}

// Visits the ids of T in ascending order, up to 64 at a time: visit(ids held by
// the lanes, count).  The scan path compacts each 64-particle window's hits into
// the low lanes with a lane permutation (no LDS).  Returns true when the segment
// was read by the scan.  (It writes no global memory, so the records the visitor
// reads stay provably unclobbered and load through the scalar cache.)
template <class Visit>
__device__ __forceinline__ bool visit_tile_ids(const FrameDev& F, int tile, int lane, const TileIds& T,
                                               Visit&& visit) {
  if (!T.scan) {
    // one visit site (the visitor is inlined once): the chunks shift down through v
    int v[kSegRegs];
#pragma unroll
    for (int c = 0; c < kSegRegs; ++c) v[c] = T.v[c];
#pragma unroll 1
    for (int c0 = 0; c0 < T.cnt; c0 += 64) {
      visit(v[0], min(64, T.cnt - c0));
#pragma unroll
      for (int c = 0; c + 1 < kSegRegs; ++c) v[c] = v[c + 1];
    }
    return false;
  }
  const int ty = tile / F.ntx, tx = tile - ty * F.ntx;
  const int x0 = tx * F.tile_w, x1 = x0 + F.tile_w - 1, y0 = ty * F.tile_h, y1 = y0 + F.tile_h - 1;
  const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int64_t p0 = 0; p0 < F.n; p0 += 64) {
    const int64_t p = p0 + lane;
    const bool hit = p < F.n && box_meets(F, p, x0, x1, y0, y1);
    const uint64_t m = __ballot(hit);
    if (!m) continue;
    // hits to lanes [0, c) in order, the others to [c, 64): a permutation
    const int c = __popcll(m);
    const int hb = __popcll(m & below);
    const int dst = hit ? hb : c + (lane - hb);
    const int mine = __builtin_amdgcn_ds_permute(dst << 2, (int)p);
    visit(mine, c);
  }
  return true;
}

// ---- F5: rasterise one tile with one 64-lane wave ------------------------------
// The tile's pixel sums live in LDS as 64-bit fixed-point integers (units of
// 2^-32 um of OPD; of 2^-32 for the absorbance).  Each particle of the tile deals
// its candidate pixels (the pixels of its record's candidate rectangle that lie in
// the tile) to the 64 lanes, 64 at a time; each lane evaluates its pixel without
// branching for the common cases -- outside, inside, one edge (the half-plane box
// filter) for a prism; the centre sample for an ellipsoid; the vertical chord for
// a habit -- and adds dn * thickness, rounded down to the fixed-point grid, to the
// pixel's LDS sum (ds_add_u64).  Integer sums do not depend on their order, so the
// canvas value -- the pixel's sum converted back to FP32 once -- is a function of
// the pixel and the particles that reach it alone: bitwise the same under every
// tiling, launch order and split of the tile's particles between workgroups.
// Each term carries at most 2^-32 of rounding (FP32 accumulation would carry
// ~1e-7 relative per add).
// The costly pixels -- a prism pixel two edges reach (the clipped-polygon area),
// an ellipsoid pixel within 2e-3 of the rim and a habit pixel next to a vertical
// face (both FP64) -- are queued as (pixel, particle) and evaluated 64 at a time
// with every lane busy, then added like the others.
// A crowded tile (a stored segment of more than kSlicePairs particles) is split
// into up to kMaxSlices slices of its segment, each rasterised by its own
// workgroup into its own sums; each slice stores its sums in a plane of the
// workspace, and the last slice to finish (a counter per tile, no waiting) adds
// the planes and writes the tile.
// The offset of a pixel centre from the particle centre is exact in FP32 (both
// are multiples of the centre's ulp and the difference is small), so the rotated
// offsets u, v carry ~1e-6 px of rounding and depend on the pixel and the
// particle alone.  ABS: the same coverage (prism) or centre thickness (ellipsoid,
// habit) also adds dmu * height times it (or dmu times the habit thickness) to
// the absorbance sums; ab = (dmu * height, dmu) of the particle.
constexpr int kQueue = 128;  // queued costly pixels per wave: 64 plus one batch of appends

// LDS of one raster wave, for a tile of `area` pixels (layout of raster_lds_bytes)
struct RasterLds {
  unsigned long long* acc;   // [area] OPD, fixed point
  unsigned long long* tacc;  // [area] absorbance (ABS), fixed point
  int* qpix;                 // [kQueue] tile pixel index of a queued pixel
  int* qpid;                 // [kQueue] its particle
};

__host__ __device__ constexpr int raster_lds_bytes(int area, bool abs) {
  return 8 * area * (abs ? 2 : 1) + 8 * kQueue;
}

__device__ __forceinline__ RasterLds raster_lds(char* base, int area, bool abs) {
  RasterLds L;
  unsigned long long* f = reinterpret_cast<unsigned long long*>(base);
  L.acc = f;
  L.tacc = f + area;
  int* q = reinterpret_cast<int*>(f + area * (abs ? 2 : 1));
  L.qpix = q;
  L.qpid = q + kQueue;
  return L;
}

// v rounded down to a multiple of 2^-32, as a two's-complement 64-bit count of
// 2^-32: the integer part floor(v) in the high word, the fraction v - floor(v)
// (exact in FP64) times 2^32, truncated, in the low word.  |v| < 2^31.
__device__ __forceinline__ unsigned long long to_fixed(float v) {
  const float fl = floorf(v);
  const unsigned lo = (unsigned)(((double)v - (double)fl) * 4294967296.0);
  return ((unsigned long long)(unsigned)(int)fl << 32) | lo;
}

// A fixed-point sum back to FP32 (via FP64: one rounding to double, one to float).
__device__ __forceinline__ float from_fixed(unsigned long long q) {
  return (float)((double)(long long)q * (1.0 / 4294967296.0));
}

struct TileGeom {
  int X0, Y0, tw, th;  // tile origin (canvas pixels) and sides
  const float4* hab_enc;
  const float4* hab_raw;
  const float4* hab_info;
  uint32_t topo_lo, topo_hi;
};

// A select the compiler keeps as v_cndmask (both operands already computed)
// rather than turning into a divergent branch.
__device__ __forceinline__ float sel(bool c, float x, float y) {
  return __builtin_unpredictable(c) ? x : y;
}

// A load through the scalar cache of a value that no work of the running kernel
// writes (the address space of kernel-constant memory; the address is the same).
__device__ __forceinline__ PRec const_load(const PRec* p) {
  typedef const __attribute__((address_space(4))) float cfloat;
  cfloat* q = (cfloat*)(p->f);
  PRec r;
#pragma unroll
  for (int k = 0; k < 32; ++k) r.f[k] = q[k];
  return r;
}

__device__ __forceinline__ void lds_add(unsigned long long* p, float v) {
  __hip_atomic_fetch_add(p, to_fixed(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Evaluates the first `count` queued costly pixels, one per lane, and adds their
// terms to the sums.
template <bool ABS, bool HAB>
__device__ __forceinline__ void flush_costly(const FrameDev& F, const TileGeom& G, const RasterLds& L, int count,
                                          int lane) {
#pragma clang fp contract(off)
  const bool valid = lane < count;
  const int pix = valid ? L.qpix[lane] : 0;
  const int pid = valid ? L.qpid[lane] : 0;
  float val = 0.0f, tval = 0.0f;
  if (valid) {
    const PRec& r = F.recs[pid];
    const int ii = G.Y0 + pix / G.tw, jj = G.X0 + pix % G.tw;
    const float kind = r.f[3];
    if (kind == 0.0f) {
      const float area = prism_clip_area(r, ii, jj);
      val = r.f[2] * area;
      if (ABS) tval = F.absr[pid].x * area;
    } else if (kind == 1.0f) {
      // h sqrt(1 - q) in FP64 with q recomputed in FP64, times dn (and dmu)
      const double qq = ellipsoid_rim_q(r, ii, jj);
      const double sq = qq < 1.0 ? sqrt(1.0 - qq) : 0.0;
      val = (float)((double)r.f[14] * (double)r.f[15] * sq);
      if (ABS) tval = (float)((double)F.absr[pid].y * (double)r.f[15] * sq);
    } else if (HAB) {
      const int k = (int)r.f[18];
      const float4 info = G.hab_info[k];
      const float tamp = info.z, inv_cell = 1.0f / info.w;
      double t = (double)r.f[15] * habit_chord64(r, G.hab_raw + k * kMaxFaces, (int)info.x, ii, jj);
      if (tamp > 0.0f && t > 0.0)
        t = fmax(t + (double)tamp * (double)value_noise((float)jj + 0.5f, (float)ii + 0.5f, inv_cell, (uint32_t)k,
                                                        G.topo_lo, G.topo_hi), 0.0);
      val = (float)((double)r.f[14] * t);
      if (ABS) tval = (float)((double)F.absr[pid].y * t);
    }
  }
  if (valid) {  // integer sums: pixels queued twice in one batch need no ordering
    lds_add(L.acc + pix, val);
    if (ABS) lds_add(L.tacc + pix, tval);
  }
}

// Appends the lanes' costly pixels to the queue (qn entries held, wave-uniform);
// evaluates a full batch of 64 when the queue holds at least that many.
template <bool ABS, bool HAB>
__device__ __forceinline__ void queue_costly(const FrameDev& F, const TileGeom& G, const RasterLds& L, bool costly,
                                             int pix, int pid, int lane, int& qn) {
  const uint64_t cm = __ballot(costly);
  if (!cm) return;
  if (costly) {
    const int slot = qn + __builtin_amdgcn_mbcnt_hi((uint32_t)(cm >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)cm, 0u));
    L.qpix[slot] = pix;
    L.qpid[slot] = pid;
  }
  qn += __popcll(cm);
  if (qn >= 64) {
    __syncthreads();
    flush_costly<ABS, HAB>(F, G, L, 64, lane);
    // keep the rest (fewer than 64) at the head of the queue
    const int rest = qn - 64;
    const int mp = lane < rest ? L.qpix[64 + lane] : 0, md = lane < rest ? L.qpid[64 + lane] : 0;
    __syncthreads();
    if (lane < rest) {
      L.qpix[lane] = mp;
      L.qpid[lane] = md;
    }
    __syncthreads();
    qn = rest;
  }
}

// Adds particle `pid` (record r, uniform) to the tile sums.
template <bool ABS, bool HAB>
__device__ __forceinline__ void raster_particle(const FrameDev& F, const TileGeom& G, const RasterLds& L,
                                                const PRec& r, int pid, int lane, int& qn) {
#pragma clang fp contract(off)
  const int jlo = max(__float_as_int(r.f[28]), G.X0), jhi = min(__float_as_int(r.f[29]), G.X0 + G.tw - 1);
  const int ilo = max(__float_as_int(r.f[30]), G.Y0), ihi = min(__float_as_int(r.f[31]), G.Y0 + G.th - 1);
  if (jlo > jhi || ilo > ihi) return;
  const int w = jhi - jlo + 1, m = w * (ihi - ilo + 1);
  const float inv_w = __builtin_amdgcn_rcpf((float)w);  // row = floor((k + 1/2) / w), exact for k < 1024
  const float kind = r.f[3];
  const float cx = r.f[0], cy = r.f[1], amp = r.f[2], c = r.f[4], s = r.f[5];
  const float2 ab = ABS ? F.absr[pid] : make_float2(0.0f, 0.0f);
  const int lx = jlo - G.X0, ly = ilo - G.Y0;
  // pixel centre offsets from the particle centre, measured from the particle's
  // own first candidate (not the tile's): dx = dx0 + (j - cj0) is then a function
  // of the pixel and the particle alone, whatever the tiling (and exact wherever
  // the centre's ulp is at least 2^-24 of the offset)
  const int cj0 = __float_as_int(r.f[28]), ci0 = __float_as_int(r.f[30]);
  const float dx0 = ((float)cj0 + 0.5f) - cx, dy0 = ((float)ci0 + 0.5f) - cy;
  const int ox = jlo - cj0, oy = ilo - ci0;
  if (kind == 0.0f) {
    const float a = r.f[6], b = r.f[7];
    // half-plane box filter constants (as in halfplane_cover; (c, s) and (s, c) share them)
    const float hp_h = r.f[24], hp_l = r.f[25], hp_rp = r.f[26], hp_r2 = r.f[27];
    const float hd = hp_h + 1e-4f;  // pixel_half_extent(c, s)
    const bool a_ok = a >= hd, b_ok = b >= hd;  // the pixel cannot reach both edges of a pair
    for (int k0 = 0; k0 < m; k0 += 64) {
      const int k = k0 + lane;
      const bool valid = k < m;
      const int row = (int)(((float)k + 0.5f) * inv_w), col = k - __mul24(row, w);
      const float dx = dx0 + (float)(ox + col), dy = dy0 + (float)(oy + row);
      const float u = __builtin_fmaf(c, dx, s * dy), v = __builtin_fmaf(c, dy, -(s * dx));
      const float du = fabsf(u) - a, dv = fabsf(v) - b;  // signed distances to the nearer edges
      const bool in_u = du < -hd, in_v = dv < -hd;
      const bool inside = in_u & in_v;
      const bool outside = (du > hd) | (dv > hd);
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
      cover = sel(inside, 1.0f, cover);
      const int pix = __mul24(ly + row, G.tw) + lx + col;
      if (valid & (inside | (edge & !outside))) {
        lds_add(L.acc + pix, amp * cover);
        if (ABS) lds_add(L.tacc + pix, ab.x * cover);
      }
      queue_costly<ABS, HAB>(F, G, L, valid & !(outside | inside | edge), pix, pid, lane, qn);
    }
  } else if (kind == 1.0f) {
    const float ia = r.f[8], ib = r.f[9];
    for (int k0 = 0; k0 < m; k0 += 64) {
      const int k = k0 + lane;
      const bool valid = k < m;
      const int row = (int)(((float)k + 0.5f) * inv_w), col = k - __mul24(row, w);
      const float dx = dx0 + (float)(ox + col), dy = dy0 + (float)(oy + row);
      const float u = __builtin_fmaf(c, dx, s * dy) * ia, v = __builtin_fmaf(c, dy, -(s * dx)) * ib;
      const float qv = u * u + v * v;
      // inside: the centre sample; within 2e-3 of the rim: queued for FP64
      const bool rim = (qv > 0.998f) & (qv < 1.002f);
      // 1 - q >= 0.002 where the value is kept, so the hardware square root
      // (within 1 ulp, no denormal scaling needed) serves
      const float sq = __builtin_amdgcn_sqrtf(fmaxf(1.0f - qv, 0.0f));
      const int pix = __mul24(ly + row, G.tw) + lx + col;
      if (valid & (qv <= 0.998f)) {
        lds_add(L.acc + pix, amp * sq);
        if (ABS) lds_add(L.tacc + pix, ab.x * sq);
      }
      queue_costly<ABS, HAB>(F, G, L, valid & rim, pix, pid, lane, qn);
    }
  } else if (HAB && kind == 2.0f) {
    // polyhedral habit: chord of the vertical ray through the pixel centre (Eq. 1),
    // times the height, plus the micro-topography where it is positive
    const int hk = (int)r.f[18];
    const float4 info = G.hab_info[hk];
    const float4* __restrict__ enc = G.hab_enc + hk * kMaxFaces;
    const int nf = (int)info.x;
    const float h = r.f[15], dn = r.f[14], tamp = info.z, inv_cell = 1.0f / info.w;
    const float ia = r.f[8], ib = r.f[9];
    for (int k0 = 0; k0 < m; k0 += 64) {
      const int k = k0 + lane;
      const bool valid = k < m;
      const int row = (int)(((float)k + 0.5f) * inv_w), col = k - __mul24(row, w);
      const float px = (float)(jlo + col) + 0.5f, py = (float)(ilo + row) + 0.5f;
      const float dx = dx0 + (float)(ox + col), dy = dy0 + (float)(oy + row);
      const float U = __builtin_fmaf(c, dx, s * dy) * ia, V = __builtin_fmaf(c, dy, -(s * dx)) * ib;
      float near;
      float t = h * habit_chord(enc, nf, U, V, &near);
      if (tamp > 0.0f && t > 0.0f)
        t = fmaxf(t + tamp * value_noise(px, py, inv_cell, (uint32_t)hk, G.topo_lo, G.topo_hi), 0.0f);
      const bool costly = valid & (near < 1e-4f);  // next to a vertical face: FP64 in the queue
      const int pix = __mul24(ly + row, G.tw) + lx + col;
      if (valid & !costly & (t != 0.0f)) {
        lds_add(L.acc + pix, dn * t);
        if (ABS) lds_add(L.tacc + pix, ab.y * t);
      }
      queue_costly<ABS, HAB>(F, G, L, costly, pix, pid, lane, qn);
    }
  }
}

// Slice `slice` of tile `tile`: particles [slice, slice + 1) * cnt / S of its
// segment (S = tile_slices; 1 unless the scan gave the tile planes), or, for a
// segment the pair list does not hold, every particle whose box meets the tile.
template <bool ABS, bool HAB>
__device__ __forceinline__ void raster_tile(const FrameDev& F, int tile, int slice, int lane, char* lds) {
#pragma clang fp contract(off)
  TileGeom G;
  G.tw = F.tile_w;
  G.th = F.tile_h;
  const int ty = tile / F.ntx, tx = tile - ty * F.ntx;
  G.X0 = tx * G.tw;
  G.Y0 = ty * G.th;
  G.hab_enc = F.hab_enc;
  G.hab_raw = F.hab_raw;
  G.hab_info = F.hab_info;
  G.topo_lo = F.topo_lo;
  G.topo_hi = F.topo_hi;
  const int area = G.tw * G.th;
  const RasterLds L = raster_lds(lds, area, ABS);
  const int start = F.tile_start[tile], end = F.tile_start[tile + 1];
  const bool stored = end <= F.pair_cap;
  int S = 1, plane = 0;
  if (stored && tile_slices(end - start) > 1) {
    plane = F.tile_plane[tile];  // -1: no planes were left for this tile
    if (plane >= 0) S = tile_slices(end - start);
  }
  for (int q = lane; q < area; q += 64) {
    L.acc[q] = 0ull;
    if (ABS) L.tacc[q] = 0ull;
  }
  int qn = 0;
  const PRec* __restrict__ recs = F.recs;
  auto visit = [&](int mine, int m) {
    // wave-uniform records through the scalar cache, the next one requested
    // before the current one is rasterised
    int pid = __builtin_amdgcn_readlane(mine, 0);
    PRec nxt = const_load(recs + pid);
    for (int k = 0; k < m; ++k) {
      const PRec cur = nxt;
      const int cpid = pid;
      if (k + 1 < m) {
        pid = __builtin_amdgcn_readlane(mine, k + 1);
        nxt = const_load(recs + pid);
      }
      raster_particle<ABS, HAB>(F, G, L, cur, cpid, lane, qn);
    }
  };
  if (stored) {
    const int cnt = end - start;
    const int a0 = start + (int)((long long)cnt * slice / S), a1 = start + (int)((long long)cnt * (slice + 1) / S);
    const int* __restrict__ pids = F.pids;
    for (int c0 = a0; c0 < a1; c0 += 64) {
      const int m = min(64, a1 - c0);
      visit(lane < m ? pids[c0 + lane] : 0, m);
    }
  } else {
    // every particle whose box meets the tile, compacted to the low lanes by a lane permutation
    const int x0 = G.X0, x1 = x0 + G.tw - 1, y0 = G.Y0, y1 = y0 + G.th - 1;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int64_t p0 = 0; p0 < F.n; p0 += 64) {
      const int64_t p = p0 + lane;
      const bool hit = p < F.n && box_meets(F, p, x0, x1, y0, y1);
      const uint64_t mk = __ballot(hit);
      if (!mk) continue;
      const int c = __popcll(mk);
      const int hb = __popcll(mk & below);
      visit(__builtin_amdgcn_ds_permute((hit ? hb : c + (lane - hb)) << 2, (int)p), c);
    }
  }
  if (qn > 0) flush_costly<ABS, HAB>(F, G, L, qn, lane);
  __syncthreads();
  if (S == 1) {
    for (int q = lane; q < area; q += 64) {
      const int i = q / G.tw, j = q - i * G.tw;
      const int64_t o = (int64_t)(G.Y0 + i) * F.W + G.X0 + j;
      F.opd[o] = from_fixed(L.acc[q]);
      if (ABS) F.tau[o] = from_fixed(L.tacc[q]);
    }
  } else {
    // this slice's sums to its plane; the last slice of the tile adds the S planes
    const size_t pl = (size_t)area * (ABS ? 2 : 1);
    unsigned long long* mine = F.planes + (size_t)(plane + slice) * pl;
    // The planes are written and read with agent-scope atomic stores and loads,
    // which the GPU keeps coherent across its XCDs without a write-back of the
    // issuing L2; the stores have completed (s_waitcnt 0) before the count is
    // raised, and the last slice reads the planes after its own count.  (A
    // release/acquire fence pair here writes back and invalidates the XCD's whole
    // L2 once per slice, which cost more than slicing saved.)
    for (int q = lane; q < area; q += 64) {
      __hip_atomic_store(mine + q, L.acc[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      if (ABS) __hip_atomic_store(mine + area + q, L.tacc[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    int last = 0;
    if (lane == 0)
      last = __hip_atomic_fetch_add(&F.tile_done[tile], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == S - 1;
    if (__builtin_amdgcn_readfirstlane(last)) {
      __atomic_signal_fence(__ATOMIC_SEQ_CST);
      unsigned long long* base = F.planes + (size_t)plane * pl;
      for (int q = lane; q < area; q += 64) {
        unsigned long long a = 0ull, t = 0ull;
        for (int k = 0; k < S; ++k) {
          a += __hip_atomic_load(base + (size_t)k * pl + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (ABS) t += __hip_atomic_load(base + (size_t)k * pl + area + q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        const int i = q / G.tw, j = q - i * G.tw;
        const int64_t o = (int64_t)(G.Y0 + i) * F.W + G.X0 + j;
        F.opd[o] = from_fixed(a);
        if (ABS) F.tau[o] = from_fixed(t);
      }
    }
  }
  if (!stored && lane == 0) atomicAdd(&F.scal[1], 1);
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
  const float il = F.inv_lambda;
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
      phase_sincos(ph[u], il, &s, &c);
      const float am = expf(-tv[u]);
      buf[t + u * kThreads] = make_float2(am * c, am * s);
    }
  } else {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
      float s, c;
      phase_sincos(ph[u], il, &s, &c);
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
  F.n = p.n; F.ld = p.ld; F.pair_cap = p.pair_cap;
  F.o = optics_args(p);
  F.phase_k = p.phase_k;
  F.inv_lambda = p.inv_lambda;
  F.recs = b.recs; F.boxes = b.boxes; F.counts = b.counts; F.scal = b.scal;
  F.tile_count = b.tile_count; F.tile_start = b.tile_start; F.cursor = b.cursor;
  F.items = b.items; F.tile_plane = b.tile_plane; F.tile_done = b.tile_done;
  F.planes = b.planes; F.plane_cap = plane_count(p.pair_cap, p.tile_h * p.tile_w);
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
