// Per-particle pixel box and raster record, shared by the forward binning and
// the adjoint (which re-derives each particle's tile range from the same box).
#pragma once

#include "osog_internal.h"

namespace osog {

// Conservative pixel box of a particle.  Only exactly rounded FP32 operations
// with no contraction, so every correct implementation reproduces it bit for bit:
//   ext = max(a,b) * 1.41421366f + 1 (prism; 1.41421366f is the float just above
//   sqrt 2, so ext covers the footprint's circumradius plus a pixel), max(a,b) + 1
//   (ellipsoid) or max(a,b) * R + 1 (polyhedral habit of bounding radius R);
//   box = [floor(c - ext), floor(c + ext)] clamped to the canvas.
// Returns false (no pairs) for a non-positive or NaN half-width, a NaN bound, a
// habit the frame does not define (R <= 0) or a box that misses the canvas.
__device__ __forceinline__ bool pixel_box(float cx, float cy, float a, float b, float shape, float R, int H,
                                          int W, int4* box) {
#pragma clang fp contract(off)
  if (!(a > 0.0f) || !(b > 0.0f)) return false;
  float m = fmaxf(a, b);
  if (shape >= 1.5f && !(R > 0.0f)) return false;
  float ext = (shape < 0.5f) ? (m * 1.41421366f + 1.0f) : (shape < 1.5f ? (m + 1.0f) : (m * R + 1.0f));
  float fx0 = floorf(cx - ext), fx1 = floorf(cx + ext);
  float fy0 = floorf(cy - ext), fy1 = floorf(cy + ext);
  if (!(fx0 <= fx1) || !(fy0 <= fy1)) return false;
  if (!(fx1 >= 0.0f) || !(fy1 >= 0.0f)) return false;
  if (!(fx0 <= (float)(W - 1)) || !(fy0 <= (float)(H - 1))) return false;
  box->x = (int)fmaxf(fx0, 0.0f);
  box->y = (int)fminf(fx1, (float)(W - 1));
  box->z = (int)fmaxf(fy0, 0.0f);
  box->w = (int)fminf(fy1, (float)(H - 1));
  return true;
}

// A pixel index from an integral float, clamped far outside any canvas (the raster
// clamps it to its tile).
__device__ __forceinline__ int pixel_index(float v) { return (int)fminf(fmaxf(v, -2.0f), 65536.0f); }

// Raster record of a valid particle (layout documented with PRec).
__device__ __forceinline__ void make_record(float cx, float cy, float ang, float a, float b, float h,
                                            float dn, float shape, float R, float habit, PRec* out) {
  PRec& r = *out;
#pragma unroll
  for (int k = 0; k < 32; ++k) r.f[k] = 0.0f;
  double cd, sd;
  sincos((double)ang, &sd, &cd);
  const float c = (float)cd, s = (float)sd;
  r.f[0] = cx; r.f[1] = cy; r.f[2] = dn * h;
  r.f[4] = c; r.f[5] = s; r.f[6] = a; r.f[7] = b;
  if (shape < 0.5f) {
    r.f[3] = 0.0f;
    const float su[4] = {-1.f, 1.f, 1.f, -1.f}, sv[4] = {-1.f, -1.f, 1.f, 1.f};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const float u = su[k] * a, v = sv[k] * b;
      r.f[8 + 2 * k] = c * u - s * v;
      r.f[9 + 2 * k] = s * u + c * v;
    }
    float xlo = r.f[8], xhi = r.f[8], ylo = r.f[9], yhi = r.f[9];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int q = (k + 1) & 3;
      r.f[16 + k] = (r.f[9 + 2 * q] - r.f[9 + 2 * k]) / (r.f[8 + 2 * q] - r.f[8 + 2 * k]);
      xlo = fminf(xlo, r.f[8 + 2 * k]); xhi = fmaxf(xhi, r.f[8 + 2 * k]);
      ylo = fminf(ylo, r.f[9 + 2 * k]); yhi = fmaxf(yhi, r.f[9 + 2 * k]);
    }
    r.f[20] = cx + xlo; r.f[21] = cx + xhi; r.f[22] = cy + ylo; r.f[23] = cy + yhi;
    // per-particle constants of the raster's pixel tests: the half-plane box
    // filter of an edge whose normal is (c, s) or (s, c) (p = max, q = min of
    // |c|, |s|), and the footprint bounds widened by half a pixel (exact shifts)
    const float p = fmaxf(fabsf(c), fabsf(s)), q = fminf(fabsf(c), fabsf(s));
    r.f[24] = 0.5f * (p + q);
    r.f[25] = 0.5f * (p - q);
    r.f[26] = __builtin_amdgcn_rcpf(p);
    r.f[27] = __builtin_amdgcn_rcpf(fmaxf(2.0f * p * q, 1e-30f));
    // candidate pixels: those whose square meets the bounds
    r.f[28] = __int_as_float(pixel_index(floorf(r.f[20])));
    r.f[29] = __int_as_float(pixel_index(ceilf(r.f[21]) - 1.0f));
    r.f[30] = __int_as_float(pixel_index(floorf(r.f[22])));
    r.f[31] = __int_as_float(pixel_index(ceilf(r.f[23]) - 1.0f));
  } else {
    r.f[3] = shape < 1.5f ? 1.0f : 2.0f;
    r.f[8] = 1.0f / a;
    r.f[9] = 1.0f / b;
    r.f[10] = __int_as_float(__double2loint(cd));
    r.f[11] = __int_as_float(__double2hiint(cd));
    r.f[12] = __int_as_float(__double2loint(sd));
    r.f[13] = __int_as_float(__double2hiint(sd));
    r.f[14] = dn;
    r.f[15] = h;
    // bounding-box half extents of the ellipse, enlarged so that every pixel centre
    // outside them has q >= 1.002 after FP32 rounding
    if (shape < 1.5f) {
      const float ex = sqrtf(a * a * c * c + b * b * s * s), ey = sqrtf(a * a * s * s + b * b * c * c);
      r.f[16] = ex * 1.0011f + 1e-3f;
      r.f[17] = ey * 1.0011f + 1e-3f;
    } else {  // habit: every point of the solid lies within max(a, b) R of the centre
      r.f[16] = fmaxf(a, b) * R * 1.0001f + 1e-3f;
      r.f[17] = r.f[16];
      r.f[18] = habit;
    }
    // candidate pixels: those whose centre lies inside the enlarged box
    r.f[28] = __int_as_float(pixel_index(ceilf((cx - r.f[16]) - 0.5f)));
    r.f[29] = __int_as_float(pixel_index(floorf((cx + r.f[16]) - 0.5f)));
    r.f[30] = __int_as_float(pixel_index(ceilf((cy - r.f[17]) - 0.5f)));
    r.f[31] = __int_as_float(pixel_index(floorf((cy + r.f[17]) - 0.5f)));
  }
}

}  // namespace osog
