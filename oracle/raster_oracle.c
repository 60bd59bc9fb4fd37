/*
 * Oracle rasteriser -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, single-threaded FP64 evaluation of the optical path difference
 * canvas: OPD[i][j] = sum_p dn_p * t_p(i, j) (paper Sec. III.A, Eq. 1, and
 * Sec. III.B, Eq. 2: the phase integral of (n_p - n_m) over the thickness; the
 * scatter-add composition of Sec. III.C, Eq. 7, is a plain sum here).
 *
 * Geometry (readings written down with the oracle's Python side):
 *   pixel (i = row, j = column) is the unit square [j, j+1] x [i, i+1];
 *   R(alpha) = [[cos, -sin], [sin, cos]] maps particle-local (u, v) to (x, y).
 *   prism    : solid {c + R(u, v) : |u| <= a, |v| <= b} of constant height h;
 *              t = h * area(pixel  intersect  footprint), the exact box filter,
 *              by Sutherland-Hodgman clipping and the shoelace formula.
 *   ellipsoid: in-plane semi-axes a, b, full central thickness h;
 *              t = h * sqrt(max(0, 1 - (u/a)^2 - (v/b)^2)) at the pixel centre.
 *
 * Only this file's plain loops compute the canvas; nothing is shared with the
 * GPU library.  Only tests, the smoke check and the CPU baseline of the
 * benchmark load it.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

typedef struct { double x, y; } pt;

/* Keep the part of the convex polygon `in` (n vertices) on one side of the
 * axis-aligned line coord(axis) = bound.  keep_ge: keep coord >= bound. */
static int clip_half(const pt* in, int n, pt* out, int axis, double bound, int keep_ge) {
  int m = 0;
  for (int k = 0; k < n; ++k) {
    pt p = in[k], q = in[(k + 1) % n];
    double cp = axis == 0 ? p.x : p.y, cq = axis == 0 ? q.x : q.y;
    int pin = keep_ge ? cp >= bound : cp <= bound;
    int qin = keep_ge ? cq >= bound : cq <= bound;
    if (pin) out[m++] = p;
    if (pin != qin) {
      double t = (bound - cp) / (cq - cp);
      pt r;
      r.x = p.x + t * (q.x - p.x);
      r.y = p.y + t * (q.y - p.y);
      if (axis == 0) r.x = bound; else r.y = bound;
      out[m++] = r;
    }
  }
  return m;
}

static double shoelace(const pt* p, int n) {
  double s = 0.0;
  for (int k = 0; k < n; ++k) {
    pt a = p[k], b = p[(k + 1) % n];
    s += a.x * b.y - b.x * a.y;
  }
  return 0.5 * s;
}

/* Area of (unit pixel [x0,x0+1] x [y0,y0+1]) intersect (convex CCW polygon). */
double oracle_pixel_area(const double* px, const double* py, int n, double x0, double y0) {
  pt a[16], b[16];
  for (int k = 0; k < n; ++k) { a[k].x = px[k]; a[k].y = py[k]; }
  int m = n;
  m = clip_half(a, m, b, 0, x0, 1);        if (m == 0) return 0.0;
  m = clip_half(b, m, a, 0, x0 + 1.0, 0);  if (m == 0) return 0.0;
  m = clip_half(a, m, b, 1, y0, 1);        if (m == 0) return 0.0;
  m = clip_half(b, m, a, 1, y0 + 1.0, 0);  if (m == 0) return 0.0;
  return shoelace(a, m);
}

static long lmax(long a, long b) { return a > b ? a : b; }
static long lmin(long a, long b) { return a < b ? a : b; }

/* Thickness-weighted OPD of one particle added into opd[H][W] (row-major).
 * soa rows: 0 cx 1 cy 2 angle 3 a 4 b 5 height 6 dn 7 shape (< 0.5 prism, < 1.5
 * ellipsoid; >= 1.5 polyhedral habits, added by the Python side, habits.py). */
static void add_particle(int H, int W, double cx, double cy, double ang, double a, double b,
                         double h, double dn, double shape, double* opd) {
  if (!(a > 0.0) || !(b > 0.0) || shape >= 1.5) return;
  double c = cos(ang), s = sin(ang);
  if (shape < 0.5) {
    /* footprint corners, counter-clockwise in the local frame */
    static const double su[4] = {-1.0, 1.0, 1.0, -1.0};
    static const double sv[4] = {-1.0, -1.0, 1.0, 1.0};
    double vx[4], vy[4], xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int k = 0; k < 4; ++k) {
      double u = su[k] * a, v = sv[k] * b;
      vx[k] = cx + c * u - s * v;
      vy[k] = cy + s * u + c * v;
      if (vx[k] < xmin) xmin = vx[k];
      if (vx[k] > xmax) xmax = vx[k];
      if (vy[k] < ymin) ymin = vy[k];
      if (vy[k] > ymax) ymax = vy[k];
    }
    if (!(xmax >= 0.0) || !(ymax >= 0.0) || !(xmin <= (double)W) || !(ymin <= (double)H)) return;
    long j0 = lmax(0, (long)floor(xmin)), j1 = lmin(W - 1, (long)floor(xmax));
    long i0 = lmax(0, (long)floor(ymin)), i1 = lmin(H - 1, (long)floor(ymax));
    for (long i = i0; i <= i1; ++i)
      for (long j = j0; j <= j1; ++j) {
        double area = oracle_pixel_area(vx, vy, 4, (double)j, (double)i);
        if (area != 0.0) opd[i * (long)W + j] += dn * h * area;
      }
  } else {
    double r = a > b ? a : b;
    if (!(cx + r >= -1.0) || !(cy + r >= -1.0) || !(cx - r <= W + 1.0) || !(cy - r <= H + 1.0)) return;
    long j0 = lmax(0, (long)floor(cx - r) - 1), j1 = lmin(W - 1, (long)floor(cx + r) + 1);
    long i0 = lmax(0, (long)floor(cy - r) - 1), i1 = lmin(H - 1, (long)floor(cy + r) + 1);
    for (long i = i0; i <= i1; ++i)
      for (long j = j0; j <= j1; ++j) {
        double dx = (double)j + 0.5 - cx, dy = (double)i + 0.5 - cy;
        double u = c * dx + s * dy, v = -s * dx + c * dy;
        double q = (u / a) * (u / a) + (v / b) * (v / b);
        if (q < 1.0) opd[i * (long)W + j] += dn * h * sqrt(1.0 - q);
      }
  }
}

/* opd[H][W] = sum over the n particles of soa[8][ld] (FP32 values widened to FP64). */
void oracle_opd(int H, int W, const float* soa, int64_t n, int64_t ld, double* opd) {
  memset(opd, 0, sizeof(double) * (size_t)H * (size_t)W);
  for (int64_t p = 0; p < n; ++p)
    add_particle(H, W, soa[0 * ld + p], soa[1 * ld + p], soa[2 * ld + p], soa[3 * ld + p],
                 soa[4 * ld + p], soa[5 * ld + p], soa[6 * ld + p], soa[7 * ld + p], opd);
}

/* Same, with the particle table already in FP64 (used by the finite-difference
 * gradients, whose steps are below FP32 resolution). */
void oracle_opd_f64(int H, int W, const double* soa, int64_t n, int64_t ld, double* opd) {
  memset(opd, 0, sizeof(double) * (size_t)H * (size_t)W);
  for (int64_t p = 0; p < n; ++p)
    add_particle(H, W, soa[0 * ld + p], soa[1 * ld + p], soa[2 * ld + p], soa[3 * ld + p],
                 soa[4 * ld + p], soa[5 * ld + p], soa[6 * ld + p], soa[7 * ld + p], opd);
}

/* OPD at a list of pixels only (for sampled comparisons at full size). */
void oracle_opd_at(int H, int W, const float* soa, int64_t n, int64_t ld,
                   const int64_t* rows, const int64_t* cols, int64_t m, double* out) {
  (void)H; (void)W;
  for (int64_t k = 0; k < m; ++k) out[k] = 0.0;
  for (int64_t p = 0; p < n; ++p) {
    double cx = soa[0 * ld + p], cy = soa[1 * ld + p], ang = soa[2 * ld + p];
    double a = soa[3 * ld + p], b = soa[4 * ld + p], h = soa[5 * ld + p];
    double dn = soa[6 * ld + p], shape = soa[7 * ld + p];
    if (!(a > 0.0) || !(b > 0.0) || shape >= 1.5) continue;
    double r = (a > b ? a : b) * 1.5 + 2.0;
    double c = cos(ang), s = sin(ang);
    for (int64_t k = 0; k < m; ++k) {
      double i = (double)rows[k], j = (double)cols[k];
      if (fabs(j + 0.5 - cx) > r || fabs(i + 0.5 - cy) > r) continue;
      if (shape < 0.5) {
        static const double su[4] = {-1.0, 1.0, 1.0, -1.0};
        static const double sv[4] = {-1.0, -1.0, 1.0, 1.0};
        double vx[4], vy[4];
        for (int q = 0; q < 4; ++q) {
          double u = su[q] * a, v = sv[q] * b;
          vx[q] = cx + c * u - s * v;
          vy[q] = cy + s * u + c * v;
        }
        out[k] += dn * h * oracle_pixel_area(vx, vy, 4, j, i);
      } else {
        double dx = j + 0.5 - cx, dy = i + 0.5 - cy;
        double u = c * dx + s * dy, v = -s * dx + c * dy;
        double q = (u / a) * (u / a) + (v / b) * (v / b);
        if (q < 1.0) out[k] += dn * h * sqrt(1.0 - q);
      }
    }
  }
}
