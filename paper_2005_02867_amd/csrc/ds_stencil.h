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

// TVD (van Leer) face value along one grid line: face f lies between cells
// f-1 and f; `line` points at cell 0 of the line, `st` is the stride.
__device__ __forceinline__ double face_value(const double* __restrict__ phi, long long line, long long st,
                                             int f, int na, double uf, double amb) {
  if (f == 0) return uf > 0.0 ? amb : phi[line];
  if (f == na) return uf < 0.0 ? amb : phi[line + (long long)(na - 1) * st];
  if (uf == 0.0) return 0.0;
  double C, D, U;
  if (uf > 0.0) {
    C = phi[line + (long long)(f - 1) * st];
    D = phi[line + (long long)f * st];
    U = (f >= 2) ? phi[line + (long long)(f - 2) * st] : C;
  } else {
    C = phi[line + (long long)f * st];
    D = phi[line + (long long)(f - 1) * st];
    U = (f + 1 <= na - 1) ? phi[line + (long long)(f + 1) * st] : C;
  }
  // van Leer: with r = (C - U)/(D - C) and psi = (r + |r|)/(1 + |r|), the face
  // value C + psi (D - C)/2 equals C + (C - U)(D - C)/(D - U) for r > 0 and C
  // otherwise -- one division instead of two.
  const double den = D - C, up = C - U;
  if (!((up > 0.0 && den > 0.0) || (up < 0.0 && den < 0.0))) return C;
  return C + up * den / (D - U);
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
