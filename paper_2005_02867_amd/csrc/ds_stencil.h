// Device helpers shared by the forward step kernels and their adjoints:
// zero-ghost alpha lookup, TVD face values, the liquid-marker face
// velocity, boundary face velocities and neighbour indices.
#pragma once
#include "ds_device.h"

namespace dsv {

__device__ __forceinline__ double alpha_or0(const DevParams& P, const double* a, int i, int j, int k) {
  if (i < 0 || j < 0 || k < 0 || i >= P.nx || j >= P.ny || k >= P.nz) return 0.0;
  return a[cidx(P, i, j, k)];
}

// TVD (van Leer) value on the interior face between cells a (lower) and b
// (upper) of a grid line, for face velocity uf; m and p are the cells beyond
// a and b, hm/hp whether they exist (else the upwind cell stands in for the
// far-upwind one).  Branch-free: the caller loads every candidate first.
// With r = (C - U)/(D - C) and psi = (r + |r|)/(1 + |r|), the face value
// C + psi (D - C)/2 equals C + (C - U)(D - C)/(D - U) for r > 0 and C
// otherwise -- one division instead of two.
__device__ __forceinline__ double tvd_face(double m, double a, double b, double p, bool hm, bool hp, double uf) {
  const bool fwd = uf > 0.0;
  const double C = fwd ? a : b, D = fwd ? b : a;
  const double U = fwd ? (hm ? m : a) : (hp ? p : b);
  const double den = D - C, up = C - U;
  const bool mono = (up > 0.0 && den > 0.0) || (up < 0.0 && den < 0.0);
  const double v = mono ? C + up * den / (D - U) : C;
  return uf == 0.0 ? 0.0 : v;
}

// Face value on a box face of a cell's line: the ambient value where the
// flow enters (uf > 0 on the low side, uf < 0 on the high side), else the
// cell's own value.
__device__ __forceinline__ double box_face(double cell, double amb, double uf, int side) {
  return (side == 0 ? uf > 0.0 : uf < 0.0) ? amb : cell;
}

// Liquid-marker face velocity: the divergence-free part u - G phi (phi = 0
// half a cell outside open faces; walls and inlets keep their value).
__device__ __forceinline__ double liquid_face_u(const DevParams& P, const double* __restrict__ phi, double uf,
                                                long long line, long long st, int f, int na, int ax) {
  if (!phi) return uf;
  if (f == 0 || f == na) {
    if (!pressure_dirichlet(P.kind[ax * 2 + (f == 0 ? 0 : 1)])) return uf;
    const double pc = phi[line + (long long)(f == 0 ? 0 : na - 1) * st];
    return f == 0 ? uf - 2.0 * pc / P.h : uf + 2.0 * pc / P.h;
  }
  return uf - (phi[line + (long long)f * st] - phi[line + (long long)(f - 1) * st]) / P.h;
}

// Boundary face velocity of cell (i,j,k) on box face (ax, side).
__device__ __forceinline__ double bface_u(const DevParams& P, const double* u, const double* v,
                                          const double* w, int ax, int side, int i, int j, int k) {
  if (ax == 0) return u[uidx(P, side ? i + 1 : i, j, k)];
  if (ax == 1) return v[vidx(P, i, side ? j + 1 : j, k)];
  return w[widx(P, i, j, side ? k + 1 : k)];
}

// Values of a at the six neighbours of cell c in the order x-, x+, y-, y+,
// z-, z+ (index ax*2 + side); has[f]: the neighbour exists.  A missing
// neighbour reads the cell itself, so all six loads are issued before any
// is used (no load waits behind a branch on the position).
__device__ __forceinline__ void nbr6(const DevParams& P, const double* __restrict__ a, long long c, int i, int j,
                                     int k, double (&o)[6], bool (&has)[6]) {
  const long long sx = (long long)P.ny * P.nz, sy = P.nz;
  has[0] = i > 0;
  has[1] = i < P.nx - 1;
  has[2] = j > 0;
  has[3] = j < P.ny - 1;
  has[4] = k > 0;
  has[5] = k < P.nz - 1;
  const long long f[6] = {has[0] ? c - sx : c, has[1] ? c + sx : c, has[2] ? c - sy : c,
                          has[3] ? c + sy : c, has[4] ? c - 1 : c,  has[5] ? c + 1 : c};
#pragma unroll
  for (int q = 0; q < 6; ++q) o[q] = a[f[q]];
}

// Neighbour of (i,j,k) across face (ax, side); returns -1 outside the box.
__device__ __forceinline__ long long nbr(const DevParams& P, int ax, int side, int i, int j, int k) {
  const int d = side ? 1 : -1;
  if (ax == 0) {
    const int ii = i + d;
    return (ii < 0 || ii >= P.nx) ? -1 : cidx(P, ii, j, k);
  }
  if (ax == 1) {
    const int jj = j + d;
    return (jj < 0 || jj >= P.ny) ? -1 : cidx(P, i, jj, k);
  }
  const int kk = k + d;
  return (kk < 0 || kk >= P.nz) ? -1 : cidx(P, i, j, kk);
}

}  // namespace dsv
