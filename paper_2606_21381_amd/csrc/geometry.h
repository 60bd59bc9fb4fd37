// Per-pixel particle thickness (paper Sec. III.A, Eq. 1 with M = 4 vertical
// side faces plus top and bottom for the prism; the ellipsoid height profile)
// and its derivatives.  Included by the raster and adjoint kernels.
#pragma once

#include "osog_internal.h"

namespace osog {

// Average of clamp(y, 0, 1) over y running linearly from y1 to y2.
// Written as (fraction of [lo,hi] inside [0,1]) * (mean inside) + (fraction
// above 1) so that short or flat segments stay well conditioned.
__device__ __forceinline__ float clamp_avg(float y1, float y2) {
#pragma clang fp contract(off)
  float lo = fminf(y1, y2), hi = fmaxf(y1, y2);
  float clo = fminf(fmaxf(lo, 0.0f), 1.0f), chi = fminf(fmaxf(hi, 0.0f), 1.0f);
  float d = hi - lo;
  if (!(d > 1e-30f)) return clo;
  const float inv = __builtin_amdgcn_rcpf(d);  // hardware reciprocal (1 ulp)
  float fin = fminf((chi - clo) * inv, 1.0f);
  float above = fmaxf(0.0f, hi - fmaxf(lo, 1.0f)) * inv;
  return fin * ((clo + chi) * 0.5f) + above;
}

// Signed contribution of the directed edge P->Q (slope sl = dy/dx) of a
// counter-clockwise polygon to its area inside the unit square [0,1]^2:
// -integral over x in [0,1] of clamp(y(x), 0, 1) dx along the edge (Green's
// theorem, area = -closed integral y dx, with y clamped to the square).
__device__ __forceinline__ float edge_area(float px, float py, float qx, float qy, float sl) {
#pragma clang fp contract(off)
  float xl = fminf(px, qx), xr = fmaxf(px, qx);
  float a = fmaxf(xl, 0.0f), b = fminf(xr, 1.0f);
  if (!(b > a)) return 0.0f;
  float ya = (a == px) ? py : ((a == qx) ? qy : py + (a - px) * sl);
  float yb = (b == px) ? py : ((b == qx) ? qy : py + (b - px) * sl);
  float w = (b - a) * clamp_avg(ya, yb);
  return (qx > px) ? -w : w;
}

// Axis-aligned bounds of a prism footprint in canvas pixels (xmin, xmax, ymin, ymax),
// rounded the same way wherever they are used.
__device__ __forceinline__ float4 prism_bounds(const PRec& r) {
  return make_float4(r.f[20], r.f[21], r.f[22], r.f[23]);
}

// Half-extent of the unit pixel along either prism axis, (|cos| + |sin|) / 2,
// plus a margin for the FP32 rounding of the rotated centre offsets (< 1e-5 px).
__device__ __forceinline__ float pixel_half_extent(float c, float s) {
  return 0.5f * (fabsf(c) + fabsf(s)) + 1e-4f;
}

// Centre-sample test of a pixel against the prism slabs: +1 when the whole pixel
// is inside (coverage exactly 1), -1 when it is certainly outside, 0 otherwise.
__device__ __forceinline__ int prism_classify(const PRec& r, float px, float py, float margin) {
#pragma clang fp contract(off)
  const float c = r.f[4], s = r.f[5], a = r.f[6], b = r.f[7];
  const float dx = px - r.f[0], dy = py - r.f[1];
  const float u = c * dx + s * dy, v = -s * dx + c * dy;
  const float hd = pixel_half_extent(c, s);
  if (fabsf(u) > a + hd || fabsf(v) > b + hd) return -1;
  if (fabsf(u) < a - hd - margin && fabsf(v) < b - hd - margin) return 1;
  return 0;
}

// Area of the unit pixel on the inner side of one straight edge: the pixel's
// box filter of a half-plane.  t = signed distance from the pixel centre to the
// edge line (positive inside), (nx, ny) = the line's unit normal.  With
// p = max(|nx|,|ny|), q = min: 0 for t <= -(p+q)/2, 1 for t >= (p+q)/2, linear
// 1/2 + t/p for |t| <= (p-q)/2 and quadratic in between.
__device__ __forceinline__ float halfplane_cover(float t, float nx, float ny) {
#pragma clang fp contract(off)
  const float p = fmaxf(fabsf(nx), fabsf(ny)), q = fminf(fabsf(nx), fabsf(ny));
  const float h = 0.5f * (p + q), l = 0.5f * (p - q);
  if (t >= h) return 1.0f;
  if (t <= -h) return 0.0f;
  if (fabsf(t) <= l) return 0.5f + t * __builtin_amdgcn_rcpf(p);
  const float e = h - fabsf(t);
  const float tri = e * e * __builtin_amdgcn_rcpf(2.0f * p * q);
  return t > 0.0f ? 1.0f - tri : tri;
}

// Area of pixel (i, j) inside the prism footprint by the clipped-polygon
// integral over its four edges (any pixel; used where two edges reach it).
// Pixel-corner offsets j - cx and i - cy are exact in FP32 for on-canvas
// particles, so the clip runs in small local coordinates.
__device__ __forceinline__ float prism_clip_area(const PRec& r, int i, int j) {
#pragma clang fp contract(off)
  const float fj = (float)j, fi = (float)i;
  const float X0 = fj - r.f[0], Y0 = fi - r.f[1];
  const float x0 = r.f[8] - X0, y0 = r.f[9] - Y0, x1 = r.f[10] - X0, y1 = r.f[11] - Y0;
  const float x2 = r.f[12] - X0, y2 = r.f[13] - Y0, x3 = r.f[14] - X0, y3 = r.f[15] - Y0;
  float area = edge_area(x0, y0, x1, y1, r.f[16]);
  area += edge_area(x1, y1, x2, y2, r.f[17]);
  area += edge_area(x2, y2, x3, y3, r.f[18]);
  area += edge_area(x3, y3, x0, y0, r.f[19]);
  return area;
}

// Exact area of pixel (i, j) covered by the prism footprint of record r (bounds
// bb from prism_bounds).  Exactly 0 for a pixel outside the bounds and exactly 1
// for a pixel inside both slabs; a single half-plane's box filter
// where only one edge reaches the pixel; otherwise the clipped polygon area.
__device__ __forceinline__ float prism_cover(const PRec& r, const float4& bb, int i, int j) {
#pragma clang fp contract(off)
  const float fj = (float)j, fi = (float)i;
  if (bb.y <= fj || bb.x >= fj + 1.0f || bb.w <= fi || bb.z >= fi + 1.0f) return 0.0f;
  const float c = r.f[4], s = r.f[5], a = r.f[6], b = r.f[7];
  const float dx = (fj + 0.5f) - r.f[0], dy = (fi + 0.5f) - r.f[1];
  const float u = c * dx + s * dy, v = -s * dx + c * dy;
  const float hd = pixel_half_extent(c, s);
  const float du = fabsf(u) - a, dv = fabsf(v) - b;  // signed distances to the nearer edges
  if (du > hd || dv > hd) return 0.0f;
  if (du < -hd && dv < -hd) return 1.0f;
  // only one pair of edges reaches the pixel, and only its nearer edge (the far
  // one is >= 2a - hd away): the pixel meets a single half-plane
  if (dv < -hd && a >= hd) return halfplane_cover(-du, c, s);
  if (du < -hd && b >= hd) return halfplane_cover(-dv, s, c);
  return prism_clip_area(r, i, j);
}

// q = (u/a)^2 + (v/b)^2 at the centre of pixel (i, j) in FP64 (used within 2e-3
// of the rim, where sqrt(1 - q) amplifies rounding).
__device__ __forceinline__ double ellipsoid_rim_q(const PRec& r, int i, int j) {
#pragma clang fp contract(off)
  const float cx = r.f[0], cy = r.f[1];
  double cd = __hiloint2double(__float_as_int(r.f[11]), __float_as_int(r.f[10]));
  double sd = __hiloint2double(__float_as_int(r.f[13]), __float_as_int(r.f[12]));
  double ddx = ((double)j + 0.5) - (double)cx, ddy = ((double)i + 0.5) - (double)cy;
  double uu = (cd * ddx + sd * ddy) / (double)r.f[6];
  double vv = (-sd * ddx + cd * ddy) / (double)r.f[7];
  return uu * uu + vv * vv;
}

// ---- polyhedral habits (Eq. 1) ------------------------------------------------
// Unit chord W_hi - W_lo (clamped at 0) of a habit's encoded faces at (U, V), FP32.
// *near: the smallest |n_x U + n_y V - d| over its vertical faces, where the
// chord jumps (a pixel that close is recomputed in FP64).
__device__ __forceinline__ float habit_chord(const float4* __restrict__ enc, int nf, float U, float V, float* near) {
#pragma clang fp contract(off)
  float lo = -__builtin_inff(), hi = __builtin_inff(), nr = __builtin_inff();
  bool ok = true;
  for (int f = 0; f < nf; ++f) {
    const float4 e = enc[f];
    const float val = __builtin_fmaf(e.x, U, __builtin_fmaf(e.y, V, e.z));
    if (e.w > 0.0f) hi = fminf(hi, val);
    else if (e.w < 0.0f) lo = fmaxf(lo, val);
    else {
      ok = ok & (val <= 0.0f);
      nr = fminf(nr, fabsf(val));
    }
  }
  *near = nr;
  return ok ? fmaxf(hi - lo, 0.0f) : 0.0f;
}

// The same chord in FP64 from the faces as given, at the centre of pixel (i, j).
__device__ __forceinline__ double habit_chord64(const PRec& r, const float4* __restrict__ raw, int nf, int i, int j) {
#pragma clang fp contract(off)
  const double cd = __hiloint2double(__float_as_int(r.f[11]), __float_as_int(r.f[10]));
  const double sd = __hiloint2double(__float_as_int(r.f[13]), __float_as_int(r.f[12]));
  const double ddx = ((double)j + 0.5) - (double)r.f[0], ddy = ((double)i + 0.5) - (double)r.f[1];
  const double U = (cd * ddx + sd * ddy) / (double)r.f[6];
  const double V = (-sd * ddx + cd * ddy) / (double)r.f[7];
  double lo = -__builtin_inff(), hi = __builtin_inff();
  bool ok = true;
  for (int f = 0; f < nf; ++f) {
    const float4 e = raw[f];
    const double c = (double)e.w - (double)e.x * U - (double)e.y * V;
    if (e.z > 0.0f) hi = fmin(hi, c / (double)e.z);
    else if (e.z < 0.0f) lo = fmax(lo, c / (double)e.z);
    else ok = ok && c >= 0.0;
  }
  return ok ? fmax(hi - lo, 0.0) : 0.0;
}

// Micro-topography value noise at canvas point (x, y): lattice values 2u - 1 from
// the first word of the Philox block at (lattice x, lattice y, habit, 3),
// smoothstep-blended.  inv_cell = 1 / cell with cell a power of two, so x * inv_cell
// and the lattice values are exact in FP32.
__device__ __forceinline__ float topo_lattice(uint32_t ix, uint32_t iy, uint32_t k, uint32_t lo, uint32_t hi) {
  const uint4 w = philox4x32_10(make_uint4(ix, iy, k, 3u), lo, hi);
  return ((float)(w.x >> 9) + 0.5f) * (1.0f / 4194304.0f) - 1.0f;
}

__device__ __forceinline__ float value_noise(float x, float y, float inv_cell, uint32_t k, uint32_t lo, uint32_t hi) {
#pragma clang fp contract(off)
  const float gx = x * inv_cell, gy = y * inv_cell;
  const float x0 = floorf(gx), y0 = floorf(gy);
  const float fx = gx - x0, fy = gy - y0;
  const uint32_t ix = (uint32_t)(int)x0, iy = (uint32_t)(int)y0;
  const float v00 = topo_lattice(ix, iy, k, lo, hi), v10 = topo_lattice(ix + 1u, iy, k, lo, hi);
  const float v01 = topo_lattice(ix, iy + 1u, k, lo, hi), v11 = topo_lattice(ix + 1u, iy + 1u, k, lo, hi);
  const float sx = fx * fx * (3.0f - 2.0f * fx), sy = fy * fy * (3.0f - 2.0f * fy);
  const float a = v00 + (v10 - v00) * sx, b = v01 + (v11 - v01) * sx;
  return a + (b - a) * sy;
}

// Ellipsoid thickness times dn at the centre of pixel (i, j) with q in FP64.
__device__ __forceinline__ float ellipsoid_rim(const PRec& r, int i, int j) {
#pragma clang fp contract(off)
  const double qq = ellipsoid_rim_q(r, i, j);
  return qq < 1.0 ? (float)((double)r.f[14] * (double)r.f[15] * sqrt(1.0 - qq)) : 0.0f;
}

// Ellipsoid thickness times dn at the centre of pixel (i, j).  Within 2e-3 of
// the rim, where sqrt(1 - q) amplifies rounding, q is recomputed in FP64.
__device__ __forceinline__ float ellipsoid_opd(const PRec& r, int i, int j) {
#pragma clang fp contract(off)
  float cx = r.f[0], cy = r.f[1], c = r.f[4], s = r.f[5];
  float dx = ((float)j + 0.5f) - cx, dy = ((float)i + 0.5f) - cy;
  float u = (c * dx + s * dy) * r.f[8], v = (-s * dx + c * dy) * r.f[9];
  float q = u * u + v * v;
  if (q >= 1.002f) return 0.0f;
  if (q > 0.998f) return ellipsoid_rim(r, i, j);
  return r.f[2] * sqrtf(1.0f - q);
}

// Half extents of an ellipse's axis-aligned bounding box, enlarged so that every
// pixel centre outside them has q >= 1.002 after FP32 rounding.
__device__ __forceinline__ float2 ellipse_extent(const PRec& r) { return make_float2(r.f[16], r.f[17]); }

}  // namespace osog
