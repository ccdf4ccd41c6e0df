// Geometry of the geometric interface advection (Section 2.1: the paper
// advects alpha with a geometric scheme, isoAdvector): a plane per surface
// cell, the area it submerges on a cell face, the volume it cuts from a cell,
// and the time integral of a face's submerged area while the plane moves.
// FP64, one cell or face per thread.
//
// Cell-local coordinates: the cell is [0, h]^3, the liquid is n.x <= s.
// The submerged area of a face is quadratic in the plane offset between the
// offsets at which the plane passes the face's corners, the cut volume of a
// cell cubic between those of its corners; both are integrated piecewise with
// Simpson's rule, which is exact for quadratics.
#pragma once
#include "ds_device.h"

namespace dsv {

constexpr double GEO_SURF_TOL = 1e-8;   // surface cells: tol < alpha < 1 - tol
constexpr double GEO_FLAT = 1e-12;      // in-face normal below this: the plane is parallel to the face

// Area of {(y, z) in [0, h]^2 : a y + b z <= sig}, a >= b >= 0.
__device__ __forceinline__ double geo_face_area(double sig, double a, double b, double h) {
  if (a < GEO_FLAT) return sig > 0.0 ? h * h : 0.0;
  if (b == 0.0) return h * fmin(fmax(sig / a, 0.0), h);
  const double zA = fmin(fmax((sig - a * h) / b, 0.0), h);   // below zA the whole row is submerged
  const double zB = fmin(fmax(sig / b, 0.0), h);             // above zB nothing is
  return h * zA + (zB - zA) * (sig - 0.5 * b * (zA + zB)) / a;
}

// The same for a face whose in-face normal components (p, q) have any sign.
__device__ __forceinline__ void geo_face_frame(double sig, double p, double q, double h, double& sh, double& a,
                                               double& b) {
  sh = sig - fmin(p, 0.0) * h - fmin(q, 0.0) * h;
  const double ap = fabs(p), aq = fabs(q);
  a = fmax(ap, aq);
  b = fmin(ap, aq);
}

// Sum of Simpson's rule over [t0, t1] split at the four break points br[]
// (clamped into the interval), for f quadratic between them.  Neighbouring
// pieces share their end value.
template <class F>
__device__ __forceinline__ double geo_simpson(F f, double t0, double t1, double (&br)[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) br[q] = fmin(fmax(br[q], t0), t1);
  // sort the four (a five-comparator network: fixed indices, no private array)
  auto cs = [](double& x, double& y) {
    const double lo = fmin(x, y), hi = fmax(x, y);
    x = lo;
    y = hi;
  };
  cs(br[0], br[1]);
  cs(br[2], br[3]);
  cs(br[0], br[2]);
  cs(br[1], br[3]);
  cs(br[1], br[2]);
  const double pts[6] = {t0, br[0], br[1], br[2], br[3], t1};
  double tot = 0.0, flo = f(t0);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    const double lo = pts[q], hi = pts[q + 1];
    const double fhi = f(hi);
    tot += (hi - lo) / 6.0 * (flo + 4.0 * f(0.5 * (lo + hi)) + fhi);
    flo = fhi;
  }
  return tot;
}

// A plane n.x <= s in the cell frame: sp = s minus the offset of the corner
// the normal points away from (so the liquid is c1 x + c2 y + c3 z <= sp over
// [0, h]^3), c1 >= c2 >= c3 the magnitudes of n's components.
struct GeoCell {
  double shift, c1, c2, c3;
};

__device__ __forceinline__ GeoCell geo_cell(const double (&n)[3], double h) {
  double c[3] = {fabs(n[0]), fabs(n[1]), fabs(n[2])};
  // descending
  if (c[0] < c[1]) { const double t = c[0]; c[0] = c[1]; c[1] = t; }
  if (c[1] < c[2]) { const double t = c[1]; c[1] = c[2]; c[2] = t; }
  if (c[0] < c[1]) { const double t = c[0]; c[0] = c[1]; c[1] = t; }
  return {(fmin(n[0], 0.0) + fmin(n[1], 0.0) + fmin(n[2], 0.0)) * h, c[0], c[1], c[2]};
}

// Volume of {c1 x + c2 y + c3 z <= sp} in [0, h]^3: the integral over x of
// the (c2, c3) face area at offset sp - c1 x.
__device__ inline double geo_frame_volume(double sp, const GeoCell& C, double h) {
  if (C.c2 < GEO_FLAT) return h * h * fmin(fmax(sp / C.c1, 0.0), h);   // a plane normal to an axis: a slab
  double br[4] = {sp / C.c1, (sp - C.c3 * h) / C.c1, (sp - C.c2 * h) / C.c1, (sp - (C.c2 + C.c3) * h) / C.c1};
  auto f = [&](double x) { return geo_face_area(sp - C.c1 * x, C.c2, C.c3, h); };
  return geo_simpson(f, 0.0, h, br);
}

// Volume of {x in [0, h]^3 : n.x <= s}.
__device__ inline double geo_cell_volume(double s, const double (&n)[3], double h) {
  const GeoCell C = geo_cell(n, h);
  return geo_frame_volume(s - C.shift, C, h);
}

// Offset s of the plane with normal n that leaves alpha h^3 of liquid in the
// cell.  In the cell frame the volume V(sp) rises from 0 at sp = 0 to h^3 at
// sp = (c1 + c2 + c3) h, and dV/dsp = (A(sp) - A(sp - c1 h)) / c1 with A the
// (c2, c3) face area.  Newton steps inside a bracket that every evaluation
// narrows; a step that would leave the bracket is a bisection.  Start, on
// the nearer side (from the full end above alpha = 1/2): the corner cut
// V = sp^3 / (6 c1 c2 c3), exact for sp <= c3 h, else the edge cut
// V = h (sp^2 - c3 h sp + c3^2 h^2 / 3) / (2 c1 c2), exact for
// c3 h <= sp <= c2 h.  Stops once the Newton step is below 1e-12 h (it is taken: the
// result is then at rounding level) or the bracket holds no double.
__device__ inline double geo_plane_offset(double alpha, const double (&n)[3], double h) {
  const GeoCell C = geo_cell(n, h);
  const double top = (C.c1 + C.c2 + C.c3) * h;
  if (C.c2 < GEO_FLAT) return C.c1 * fmin(fmax(alpha, 0.0), 1.0) * h + C.shift;   // a slab
  const double target = alpha * h * h * h;
  double lo = 0.0, hi = top;
  const double m = fmax(alpha <= 0.5 ? alpha : 1.0 - alpha, 0.0);
  double x = cbrt(6.0 * C.c1 * C.c2 * C.c3 * m) * h;
  if (!(x < C.c3 * h)) x = 0.5 * C.c3 * h + sqrt(fmax(2.0 * C.c1 * C.c2 * m - C.c3 * C.c3 / 12.0, 0.0)) * h;
  double sp = alpha <= 0.5 ? x : top - x;
  if (!(sp > lo && sp < hi)) sp = 0.5 * (lo + hi);
  for (int it = 0; it < 100; ++it) {
    const double F = geo_frame_volume(sp, C, h) - target;
    if (F > 0.0) hi = sp;
    else if (F < 0.0) lo = sp;
    else break;
    const double dV = (geo_face_area(sp, C.c2, C.c3, h) - geo_face_area(sp - C.c1 * h, C.c2, C.c3, h)) / C.c1;
    const double d = F / dV;   // NaN or infinite where dV = 0: the comparisons below fail
    if (fabs(d) <= 1e-12 * h) {
      sp = fmin(fmax(sp - d, lo), hi);
      break;
    }
    double nx = sp - d;
    if (!(nx > lo && nx < hi)) nx = 0.5 * (lo + hi);
    if (nx == lo || nx == hi) break;   // no double left inside the bracket
    sp = nx;
  }
  return sp + C.shift;
}

// int_0^dt of the submerged area of a face (in-face normal components p, q)
// whose plane offset moves as sig0 + un t.
__device__ inline double geo_swept_area(double sig0, double un, double p, double q, double h, double dt) {
  double sh, a, b;
  geo_face_frame(sig0, p, q, h, sh, a, b);
  if (a < GEO_FLAT) {   // parallel to the face: wholly submerged while the offset is positive
    double wet;
    if (un > 0.0) wet = dt - fmin(fmax(-sh / un, 0.0), dt);
    else if (un < 0.0) wet = fmin(fmax(-sh / un, 0.0), dt);
    else wet = sh > 0.0 ? dt : 0.0;
    return h * h * wet;
  }
  double br[4] = {-1.0, -1.0, -1.0, -1.0};
  if (un != 0.0) {
    br[0] = (0.0 - sh) / un;
    br[1] = (b * h - sh) / un;
    br[2] = (a * h - sh) / un;
    br[3] = ((a + b) * h - sh) / un;
  }
  auto f = [&](double t) { return geo_face_area(sh + un * t, a, b, h); };
  return geo_simpson(f, 0.0, dt, br);
}

}  // namespace dsv
