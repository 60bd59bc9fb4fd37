// The forward renderer's stages as workgroup-level device bodies over a device
// frame descriptor.  The single-frame kernels (bin.hip, raster.hip, fft.hip)
// call these; the batch graph (batch.hip) replays those kernels, so a frame
// rendered alone or inside a batch goes through identical arithmetic.
//
// Every body is executed by one 256-thread workgroup (the raster body by one
// 64-lane wave) and receives a pointer to LDS scratch of at least kStageLds
// bytes; bodies that synchronise call __syncthreads() uniformly.
#pragma once

#include "bin_common.h"
#include "fft_common.h"
#include "geometry.h"
#include "osog_internal.h"

namespace osog {

// LDS one stage body may use: the largest is pass 3 at RB * W = 8192 points
// plus a 256-entry double reduction array.
constexpr int kStageLds = 8192 * 8 + kThreads * 8;  // >= pass3_buf_bytes(W) + kThreads * 8 for every W

// Everything a stage needs to know about one frame, in device-readable form.
struct FrameDev {
  int H, W, logH, logW, tile_h, tile_w, ntx, n_tiles;
  int d1, d2, nsl, nblk;          // radix digit widths, slice capacity, particle blocks
  int fft_radix;                   // FFT plan: largest Stockham radix (8 or 4)
  int64_t n, ld, cap;
  OpticsArgs o;
  float phase_k;
  const float* soa;
  const float* globals;
  float* opd;                      // caller's or workspace OPD canvas
  float* intensity;
  PRec* recs;
  int4* boxes;
  int* counts;
  long long* blocksum;
  long long* emit_start;
  int* scal;                       // [0] pairs, [1] overflow, [2] noise scale (float bits)
  int* keys_a; int* vals_a; int* keys_b; int* vals_b;
  int* hist1; int* hist2; int* dtot;
  int* tile_first; int* tile_end;
  int* sorted_vals;                // where the final radix pass leaves the particle ids
  float2* band;
  double* colsum;
};

// ---- F1: records, pixel boxes, pair counts; clears later accumulators ---------
__device__ __forceinline__ void prepare_body(const FrameDev& F, int blk, int nblocks, char* lds) {
  long long* red = reinterpret_cast<long long*>(lds);
  const int t = threadIdx.x;
  const int64_t p = (int64_t)blk * kThreads + t;
  const int64_t gsz = (int64_t)nblocks * kThreads;
  const int64_t n1 = F.d1 > 0 ? ((int64_t)1 << F.d1) * F.nsl : 0;
  const int64_t n2 = F.d2 > 0 ? ((int64_t)1 << F.d2) * F.nsl : 0;
  for (int64_t q = p; q < n1; q += gsz) F.hist1[q] = 0;
  for (int64_t q = p; q < n2; q += gsz) F.hist2[q] = 0;
  for (int64_t q = p; q < F.n_tiles; q += gsz) {
    F.tile_end[q] = 0;
    F.tile_first[q] = INT_MAX;
  }
  int cnt = 0;
  if (p < F.n) {
    const float* soa = F.soa;
    const int64_t ld = F.ld;
    const float cx = soa[0 * ld + p], cy = soa[1 * ld + p], ang = soa[2 * ld + p];
    const float a = soa[3 * ld + p], b = soa[4 * ld + p], h = soa[5 * ld + p];
    const float dn = soa[6 * ld + p], shape = soa[7 * ld + p];
    int4 box;
    const bool ok = pixel_box(cx, cy, a, b, shape, F.H, F.W, &box);
    PRec r;
#pragma unroll
    for (int k = 0; k < 32; ++k) r.f[k] = 0.0f;
    if (ok) {
      const int tx0 = box.x / F.tile_w, tx1 = box.y / F.tile_w, ty0 = box.z / F.tile_h, ty1 = box.w / F.tile_h;
      cnt = (tx1 - tx0 + 1) * (ty1 - ty0 + 1);
      make_record(cx, cy, ang, a, b, h, dn, shape, &r);
    } else {
      r.f[3] = -1.0f;
      box = make_int4(1, 0, 1, 0);
    }
    F.recs[p] = r;
    F.boxes[p] = box;
    F.counts[p] = cnt;
  }
  red[t] = cnt;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) F.blocksum[blk] = red[0];
  __syncthreads();
}

// ---- F2/F3: offsets, emission, the first radix histogram ----------------------
// hist1[d * nsl + s] = number of emitted keys with low digit d in 256-key slice s.
__device__ __forceinline__ void emit_body(const FrameDev& F, int blk, char* lds) {
  long long* red = reinterpret_cast<long long*>(lds);
  long long* scan = red + kThreads;
  const int t = threadIdx.x;
  long long pre = 0, tot = 0;
  for (int b = t; b < F.nblk; b += kThreads) {
    const long long v = F.blocksum[b];
    tot += v;
    if (b < blk) pre += v;
  }
  red[t] = pre;
  scan[t] = tot;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) { red[t] += red[t + s]; scan[t] += scan[t + s]; }
    __syncthreads();
  }
  const long long base = red[0], total = scan[0];
  const bool overflow = total > F.cap;
  if (blk == 0 && t == 0) {
    F.scal[0] = overflow ? 0 : (int)total;
    F.scal[1] = overflow ? 1 : 0;
    F.emit_start[F.n] = total;
  }
  __syncthreads();
  const int64_t p = (int64_t)blk * kThreads + t;
  const int c = p < F.n ? F.counts[p] : 0;
  scan[t] = c;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    long long v = t >= off ? scan[t - off] : 0;
    __syncthreads();
    scan[t] += v;
    __syncthreads();
  }
  long long e = base + scan[t] - c;
  if (p < F.n) F.emit_start[p] = e;
  if (!overflow && c > 0) {
    const int4 box = F.boxes[p];
    const int tx0 = box.x / F.tile_w, tx1 = box.y / F.tile_w, ty0 = box.z / F.tile_h, ty1 = box.w / F.tile_h;
    const int mask = (1 << F.d1) - 1;
    for (int ty = ty0; ty <= ty1; ++ty)
      for (int tx = tx0; tx <= tx1; ++tx) {
        const int key = ty * F.ntx + tx;
        F.keys_a[e] = key;
        F.vals_a[e] = (int)p;
        if (F.d1 > 0) {
          atomicAdd(&F.hist1[(size_t)(key & mask) * F.nsl + (e >> 8)], 1);
        } else {  // a single tile: the emission order is already sorted
          atomicMin(&F.tile_first[key], (int)e);
          atomicMax(&F.tile_end[key], (int)e + 1);
        }
        ++e;
      }
  }
  __syncthreads();
}

// ---- per-digit exclusive prefix over slices (in place), digit totals ---------
__device__ __forceinline__ void digit_offsets_body(const FrameDev& F, int pass, int d, char* lds) {
  int* part = reinterpret_cast<int*>(lds);
  const int t = threadIdx.x;
  if (F.scal[1]) return;
  int* hist = pass == 0 ? F.hist1 : F.hist2;
  int* dtot = F.dtot + (pass == 0 ? 0 : 256);
  const int nslice = (F.scal[0] + kThreads - 1) / kThreads;
  int* row = hist + (size_t)d * F.nsl;
  const int per = (nslice + kThreads - 1) / kThreads;
  const int b0 = min(nslice, t * per), b1 = min(nslice, b0 + per);
  int s = 0;
  for (int b = b0; b < b1; ++b) s += row[b];
  part[t] = s;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    int v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int run = part[t] - s;
  for (int b = b0; b < b1; ++b) {
    const int v = row[b];
    row[b] = run;
    run += v;
  }
  if (t == kThreads - 1) dtot[d] = part[t];
  __syncthreads();
}

// ---- F4: one stable scatter pass on 256-key slice `blk` -----------------------
// Per-digit output base = (exclusive scan over digits of the digit totals) +
// (exclusive prefix of the digit over earlier slices).  Keys are ranked in input
// order inside the slice (ballot-matched peers within a wave, per-wave counts
// across waves), so the sort is stable.  Pass 0 of two counts the next digit per
// output slice; the final pass marks each tile's first and one-past-last index
// (run boundaries only).  Returns without touching LDS when the slice is empty.
__device__ __forceinline__ void scatter_body(const FrameDev& F, int pass, int blk, char* lds) {
  int* base = reinterpret_cast<int*>(lds);
  int* wcnt = base + 256;  // [4][256]
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  if (F.scal[1]) return;
  const int P = F.scal[0];
  const int lo = blk * kThreads;
  if (lo >= P) return;
  const bool final_pass = (pass == 1) || F.d2 == 0;
  const int shift = pass == 0 ? 0 : F.d1, bits = pass == 0 ? F.d1 : F.d2;
  const int* kin = pass == 0 ? F.keys_a : F.keys_b;
  const int* vin = pass == 0 ? F.vals_a : F.vals_b;
  int* kout = pass == 0 ? F.keys_b : F.keys_a;
  int* vout = pass == 0 ? F.vals_b : F.vals_a;
  const int* hist = pass == 0 ? F.hist1 : F.hist2;
  const int* dtot = F.dtot + (pass == 0 ? 0 : 256);
  const int hi = min(P, lo + kThreads);
  const int nd = 1 << bits, mask = nd - 1;
  const int tot = t < nd ? dtot[t] : 0;
  base[t] = tot;
#pragma unroll
  for (int w = 0; w < kThreads / 64; ++w) wcnt[w * 256 + t] = 0;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {
    int v = t >= off ? base[t - off] : 0;
    __syncthreads();
    base[t] += v;
    __syncthreads();
  }
  const int excl = (t < nd) ? base[t] - tot + hist[(size_t)t * F.nsl + blk] : 0;
  __syncthreads();
  base[t] = excl;
  __syncthreads();
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int q = lo + t;
  const bool valid = q < hi;
  int key = 0, val = 0;
  unsigned d = 0;
  if (valid) {
    key = kin[q];
    val = vin[q];
    d = (key >> shift) & mask;
  }
  unsigned long long peers = __ballot(valid);
  for (int bit = 0; bit < bits; ++bit) {
    const bool on = (d >> bit) & 1u;
    const unsigned long long m = __ballot(on);
    peers &= on ? m : ~m;
  }
  if (!valid) peers = 0;
  const int rank = __popcll(peers & lt);
  if (valid && rank == 0) wcnt[wave * 256 + d] = __popcll(peers);
  __syncthreads();
  if (valid) {
    int off = base[d] + rank;
    for (int w = 0; w < wave; ++w) off += wcnt[w * 256 + d];
    kout[off] = key;
    vout[off] = val;
    if (final_pass) {
      // peers with one digit keep input (low-digit) order, so equal keys are
      // adjacent among them: a tile run starts/ends where the neighbouring peer differs
      const unsigned long long before = peers & lt, after = peers & ~lt & ~(1ull << lane);
      const int prev_lane = before ? 63 - __clzll(before) : -1;
      const int next_lane = after ? __ffsll(after) - 1 : -1;
      const int prev_key = __shfl(key, prev_lane < 0 ? lane : prev_lane);
      const int next_key = __shfl(key, next_lane < 0 ? lane : next_lane);
      if (prev_lane < 0 || prev_key != key) atomicMin(&F.tile_first[key], off);
      if (next_lane < 0 || next_key != key) atomicMax(&F.tile_end[key], off + 1);
    } else {
      atomicAdd(&F.hist2[(size_t)((key >> F.d1) & ((1 << F.d2) - 1)) * F.nsl + (off >> 8)], 1);
    }
  }
  __syncthreads();
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

// Contribution of one particle to one pixel of a 64-pixel slot, with the
// slot-level shortcuts (both give exactly what the per-pixel code would).
__device__ __forceinline__ float contribution(const PRec& r, const SubRect& R, int i, int j) {
#pragma clang fp contract(off)
  const float kind = r.f[3];
  if (kind == 0.0f) {
    if (r.f[21] <= R.x0 || r.f[20] >= R.x1 || r.f[23] <= R.y0 || r.f[22] >= R.y1) return 0.0f;
    // every pixel centre of the slot deep inside both slabs: coverage 1 everywhere
    // (max |u| over the rectangle of centres = |u at its middle| + |c| hx + |s| hy)
    const float c = r.f[4], s = r.f[5];
    const float hx = 0.5f * (R.x1 - R.x0 - 1.0f), hy = 0.5f * (R.y1 - R.y0 - 1.0f);
    const float dx = 0.5f * (R.x0 + R.x1) - r.f[0], dy = 0.5f * (R.y0 + R.y1) - r.f[1];
    const float ux = fabsf(c * dx + s * dy) + fabsf(c) * hx + fabsf(s) * hy;
    const float vy = fabsf(-s * dx + c * dy) + fabsf(s) * hx + fabsf(c) * hy;
    const float lim = 0.70712f + 1e-4f;
    if (ux < r.f[6] - lim && vy < r.f[7] - lim) return r.f[2];
    return r.f[2] * prism_cover(r, make_float4(r.f[20], r.f[21], r.f[22], r.f[23]), i, j);
  }
  if (kind == 1.0f) {
    if (R.x1 - 0.5f - r.f[0] < -r.f[16] || R.x0 + 0.5f - r.f[0] > r.f[16] || R.y1 - 0.5f - r.f[1] < -r.f[17] ||
        R.y0 + 0.5f - r.f[1] > r.f[17])
      return 0.0f;
    return ellipsoid_opd(r, i, j);
  }
  return 0.0f;
}

// Lane `lane` of the wave owns pixels lane, lane+64, lane+128, lane+192 of the
// tile.  The particle loop, the record load (scalar cache) and the kind dispatch
// run once per (tile, particle); ids are fetched 64 at a time and broadcast.
__device__ __forceinline__ void raster_tile(const FrameDev& F, int tile, int lane) {
#pragma clang fp contract(off)
  const int tile_w = F.tile_w, tile_h = F.tile_h;
  const int ty = tile / F.ntx, tx = tile - ty * F.ntx;
  int pi[4], pj[4];
  SubRect R[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const int q = lane + 64 * k, li = q / tile_w, lj = q - li * tile_w;
    pi[k] = ty * tile_h + li;
    pj[k] = tx * tile_w + lj;
    R[k] = slot_rect(64 * k, tile_w, tx, ty, tile_h);
  }
  float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  const PRec* __restrict__ recs = F.recs;
  if (!F.scal[1]) {
    const int start = F.tile_first[tile];
    const int cnt = max(0, F.tile_end[tile] - start);
    const int* __restrict__ pids = F.sorted_vals;
    for (int c0 = 0; c0 < cnt; c0 += 64) {
      const int m = min(64, cnt - c0);
      const int mine = lane < m ? pids[start + c0 + lane] : 0;
      PRec nxt = recs[__builtin_amdgcn_readlane(mine, 0)];
      for (int k = 0; k < m; ++k) {
        const PRec cur = nxt;
        if (k + 1 < m) nxt = recs[__builtin_amdgcn_readlane(mine, k + 1)];
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[q] += contribution(cur, R[q], pi[q], pj[q]);
      }
    }
  } else {
    // The pair list overflowed its capacity: visit every particle in id order and
    // keep those whose pixel box meets this tile (same records, same order, same sums).
    const int x0 = tx * tile_w, x1 = x0 + tile_w - 1, y0 = ty * tile_h, y1 = y0 + tile_h - 1;
    for (int64_t p = 0; p < F.n; ++p) {
      const int4 b = F.boxes[p];
      if (b.x > b.y || b.x > x1 || b.y < x0 || b.z > y1 || b.w < y0) continue;
      const PRec r = recs[p];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += contribution(r, R[q], pi[q], pj[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) F.opd[(int64_t)pi[q] * F.W + pj[q]] = acc[q];
}

// ---- F6: pass 1, rows --------------------------------------------------------
template <int LOGW, int MAXR>
__device__ __forceinline__ void pass1_body(const FrameDev& F, int rb, const float2* __restrict__ tw, char* lds) {
#pragma clang fp contract(off)
  constexpr int W = 1 << LOGW, RB = rows_per_block(W);
  float2* buf = reinterpret_cast<float2*>(lds);
  const int t = threadIdx.x;
  const float* src = F.opd + (size_t)rb * RB * W;
  const float pk = F.phase_k;
  for (int idx = t; idx < RB * W; idx += kThreads) {
    float s, c;
    sincosf(pk * src[idx], &s, &c);
    buf[idx] = make_float2(c, s);
  }
  __syncthreads();
  Stages<W, RB, -1, 1, LOGW, MAXR>::run(buf, tw);
  const int kx_lo = F.o.kx_lo, kx_n = F.o.kx_n;
  float2* dst = F.band + (size_t)rb * kx_n * RB;
  for (int idx = t; idx < kx_n * RB; idx += kThreads) {
    const int b = idx / RB, r = idx - b * RB;
    dst[idx] = buf[r * W + ((kx_lo + b) & (W - 1))];
  }
  __syncthreads();
}

// ---- F7: pass 2, one in-band column ------------------------------------------
template <int LOGH, int MAXR>
__device__ __forceinline__ void pass2_body(const FrameDev& F, int b, const float2* __restrict__ tw, char* lds) {
#pragma clang fp contract(off)
  constexpr int H = 1 << LOGH;
  float2* buf = reinterpret_cast<float2*>(lds);
  double* red = reinterpret_cast<double*>(lds + H * sizeof(float2));
  int* chord = reinterpret_cast<int*>(lds + H * sizeof(float2) + kThreads * sizeof(double));
  const OpticsArgs& o = F.o;
  const int t = threadIdx.x, kx = o.kx_lo + b;
  const int RB = o.rb;
  float2* band = F.band;
  for (int i = t; i < H; i += kThreads) buf[i] = band[((size_t)(i / RB) * o.kx_n + b) * RB + (i % RB)];
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
  red[t] = part;
  __syncthreads();
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    if (t < s) red[t] += red[t + s];
    __syncthreads();
  }
  if (t == 0) F.colsum[b] = red[0];
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
  return rows_per_block(W) * W * 8 > kNoiseQueueBytes ? rows_per_block(W) * W * 8 : kNoiseQueueBytes;
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
    __syncthreads();
    for (int q = lane; q < total; q += 64) {
      const uint4 en = queue[q];
      const int k = poisson_large(__uint_as_float(en.y), en.z, en.w, en.x, o.frame, o.seed_lo, o.seed_hi);
      queue[q].y = (uint32_t)k;
    }
    __syncthreads();
    pos = incl - cnt;
#pragma unroll
    for (int e = 0; e < 2 * CH; ++e)
      if (pend & (1u << e)) res[e] = (float)(int)queue[pos++].y;
#pragma unroll
    for (int c = 0; c < CH; ++c) {
      const int ml = t + kThreads * (k0 + c);
      if (ml < NP) out[ml] = make_float2(res[2 * c] / scale, res[2 * c + 1] / scale);
    }
    __syncthreads();  // the queue is reused by the next round
  }
}

template <int LOGW, int MAXR>
__device__ __forceinline__ void pass3_body(const FrameDev& F, int rb, const float2* __restrict__ tw, char* lds) {
#pragma clang fp contract(off)
  constexpr int W = 1 << LOGW, RB = rows_per_block(W), NP = RB * W / 2;
  constexpr int PP = (NP + kThreads - 1) / kThreads;
  float2* buf = reinterpret_cast<float2*>(lds);
  double* red = reinterpret_cast<double*>(lds + pass3_buf_bytes(W));
  const OpticsArgs& o = F.o;
  const int t = threadIdx.x;
  for (int idx = t; idx < RB * W; idx += kThreads) buf[idx] = make_float2(0.0f, 0.0f);
  __syncthreads();
  const float2* src = F.band + (size_t)rb * o.kx_n * RB;
  for (int idx = t; idx < o.kx_n * RB; idx += kThreads) {
    const int b = idx / RB, r = idx - b * RB;
    buf[r * W + ((o.kx_lo + b) & (W - 1))] = src[idx];
  }
  const bool noise = o.photons > 0.0f;
  if (noise) {
    double s = 0.0;
    for (int b = t; b < o.kx_n; b += kThreads) s += F.colsum[b];
    red[t] = s;
  }
  __syncthreads();
  float scale = 0.0f;
  if (noise) {
    for (int s = kThreads / 2; s > 0; s >>= 1) {
      if (t < s) red[t] += red[t + s];
      __syncthreads();
    }
    const double hw = (double)o.H * (double)W;
    const double mean = red[0] / (hw * hw);
    scale = mean > 0.0 ? (float)((double)o.photons / mean) : 0.0f;
  }
  Stages<W, RB, 1, 1, LOGW, MAXR>::run(buf, tw);
  const float inv = o.inv_hw;
  float* dst = F.intensity + (size_t)rb * RB * W;
  if (!(scale > 0.0f)) {
    for (int idx = t; idx < RB * W; idx += kThreads) {
      const float2 e = buf[idx];
      const float er = e.x * inv, ei = e.y * inv;
      dst[idx] = er * er + ei * ei;
    }
    __syncthreads();
    return;
  }
  // intensities of this thread's pixel pairs (ml = t + 256 k), then the LDS is free
  float Ipix[2 * PP];
#pragma unroll
  for (int k = 0; k < PP; ++k) {
    const int ml = t + kThreads * k;
#pragma unroll
    for (int x = 0; x < 2; ++x) {
      float v = 0.0f;
      if (ml < NP) {
        const float2 e = buf[2 * ml + x];
        const float er = e.x * inv, ei = e.y * inv;
        v = er * er + ei * ei;
      }
      Ipix[2 * k + x] = v;
    }
  }
  __syncthreads();
  noise_rows<NP>(F, scale, (int64_t)rb * RB * W, Ipix, dst, lds);
}

}  // namespace osog

namespace osog {

// Host: device descriptor of a planned frame on its carved workspace.  The
// caller sets soa / globals / opd / intensity.
inline FrameDev make_dev(const FramePlan& p, const FrameBufs& b) {
  FrameDev F{};
  F.H = p.H; F.W = p.W; F.logH = p.logH; F.logW = p.logW;
  F.tile_h = p.tile_h; F.tile_w = p.tile_w; F.ntx = p.ntx; F.n_tiles = p.n_tiles;
  F.d1 = (p.key_bits + 1) / 2;
  F.d2 = p.key_bits - F.d1;
  F.nsl = (int)((p.cap + kThreads - 1) / kThreads);
  F.nblk = (int)((p.n + kThreads - 1) / kThreads);
  F.n = p.n; F.ld = p.ld; F.cap = p.cap;
  F.o = optics_args(p);
  F.phase_k = p.phase_k;
  F.recs = b.recs; F.boxes = b.boxes; F.counts = b.counts; F.blocksum = b.blocksum;
  F.emit_start = b.emit_start; F.scal = b.scal;
  F.keys_a = b.keys_a; F.vals_a = b.vals_a; F.keys_b = b.keys_b; F.vals_b = b.vals_b;
  F.hist1 = b.hist1; F.hist2 = b.hist2; F.dtot = b.dtot;
  F.tile_first = b.tile_first; F.tile_end = b.tile_end;
  // two passes end in a (a -> b -> a), one pass in b, none (one tile) in a
  F.sorted_vals = (F.d1 > 0 && F.d2 == 0) ? b.vals_b : b.vals_a;
  F.band = b.band; F.colsum = b.colsum;
  F.fft_radix = p.fft_radix;
  F.opd = b.opd;
  return F;
}

}  // namespace osog
