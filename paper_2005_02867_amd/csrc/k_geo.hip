// Geometric interface advection (advection = 1; Section 2.1, eq. 3): the
// liquid fluxes of the step from a plane per surface cell.
//   k_plic: per surface cell (tol < alpha1 < 1 - tol) the plane n.x = s,
//     n = -grad(alpha1)/|grad(alpha1)| by central differences (a ghost outside
//     the box repeats its neighbour), s leaving alpha1 h^3 of liquid; only
//     surface cells are written (n = 0 where the gradient vanishes);
//   k_geo_flux: per face, the liquid volume through it in the step divided by
//     h^2 dt: the face velocity that moves the liquid (u - G phi, phi = 0
//     half a cell outside open faces, or u itself) times the time integral of
//     the area the donor (upwind) cell's plane submerges while it moves along
//     n with the donor's centre velocity; a donor that is not a surface cell,
//     or has no plane, gives U_f alpha1; inflow through a box face carries no
//     liquid.
// Both walk the cells with a grid stride, so the thin shell of surface cells,
// where the work is, is dealt over every block.
// k_advect then takes these fluxes in place of its flux-limited liquid flux.
#include <hip/hip_runtime.h>

#include "ds_device.h"
#include "ds_geo.h"
#include "ds_kernels.h"
#include "ds_stencil.h"

namespace dsv {

namespace {

__global__ void __launch_bounds__(BLOCK) k_plic(DevParams P, const double* __restrict__ a1, double* __restrict__ pnx,
                       double* __restrict__ pny, double* __restrict__ pnz, double* __restrict__ ps) {
  const double h = P.h;
  const long long stride = (long long)gridDim.x * BLOCK;
  for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < P.n; c += stride) {
    const double a = a1[c];
    if (a > GEO_SURF_TOL && a < 1.0 - GEO_SURF_TOL) {
      double n[3] = {0.0, 0.0, 0.0}, s = 0.0;
      int i, j, k;
      decode(P, c, i, j, k);
      auto at = [&](int ii, int jj, int kk) {
        return a1[cidx(P, min(max(ii, 0), P.nx - 1), min(max(jj, 0), P.ny - 1), min(max(kk, 0), P.nz - 1))];
      };
      const double gx = (at(i + 1, j, k) - at(i - 1, j, k)) / (2.0 * h);
      const double gy = (at(i, j + 1, k) - at(i, j - 1, k)) / (2.0 * h);
      const double gz = (at(i, j, k + 1) - at(i, j, k - 1)) / (2.0 * h);
      const double gm = sqrt(gx * gx + gy * gy + gz * gz);
      if (gm > 0.0) {
        n[0] = -gx / gm;
        n[1] = -gy / gm;
        n[2] = -gz / gm;
        s = geo_plane_offset(a, n, h);
      }
      pnx[c] = n[0];
      pny[c] = n[1];
      pnz[c] = n[2];
      ps[c] = s;
    }
  }
}

// Velocity that moves the liquid through face f of axis AX at cell (i, j, k)
// (f = i, j or k along AX).
template <int AX>
__device__ __forceinline__ double geo_liquid_u(const DevParams& P, const double* const (&U)[3],
                                               const double* __restrict__ phi, int i, int j, int k) {
  if (AX == 0)
    return liquid_face_u(P, phi, U[0][uidx(P, i, j, k)], (long long)j * P.nz + k, (long long)P.ny * P.nz, i, P.nx, 0);
  if (AX == 1)
    return liquid_face_u(P, phi, U[1][vidx(P, i, j, k)], (long long)i * P.ny * P.nz + k, P.nz, j, P.ny, 1);
  return liquid_face_u(P, phi, U[2][widx(P, i, j, k)], ((long long)i * P.ny + j) * P.nz, 1, k, P.nz, 2);
}

// Liquid flux density (volume / (h^2 dt)) through face f of axis AX, the face
// between cells f-1 and f along AX at the other indices (o1, o2).
template <int AX>
__device__ __forceinline__ double geo_face(const DevParams& P, const double* __restrict__ a1,
                                           const double* const (&U)[3], const double* __restrict__ phi,
                                           const double* const (&pl)[4], int i, int j, int k) {
  const int fpos = AX == 0 ? i : (AX == 1 ? j : k);
  const int nax = AX == 0 ? P.nx : (AX == 1 ? P.ny : P.nz);
  const double uf = geo_liquid_u<AX>(P, U, phi, i, j, k);
  if (uf == 0.0) return 0.0;
  const bool fwd = uf > 0.0;
  if (fwd ? fpos == 0 : fpos == nax) return 0.0;   // inflow through a box face
  int d[3] = {i, j, k};
  if (fwd) d[AX] -= 1;
  const long long dc = cidx(P, d[0], d[1], d[2]);
  const double ad = a1[dc];
  if (!(ad > GEO_SURF_TOL && ad < 1.0 - GEO_SURF_TOL)) return uf * ad;
  const double n[3] = {pl[0][dc], pl[1][dc], pl[2][dc]};
  if (n[0] == 0.0 && n[1] == 0.0 && n[2] == 0.0) return uf * ad;
  // the donor's centre velocity and the plane's normal speed
  const double uc[3] = {0.5 * (geo_liquid_u<0>(P, U, phi, d[0], d[1], d[2]) +
                               geo_liquid_u<0>(P, U, phi, d[0] + 1, d[1], d[2])),
                        0.5 * (geo_liquid_u<1>(P, U, phi, d[0], d[1], d[2]) +
                               geo_liquid_u<1>(P, U, phi, d[0], d[1] + 1, d[2])),
                        0.5 * (geo_liquid_u<2>(P, U, phi, d[0], d[1], d[2]) +
                               geo_liquid_u<2>(P, U, phi, d[0], d[1], d[2] + 1))};
  const double un = uc[0] * n[0] + uc[1] * n[1] + uc[2] * n[2];
  const double h = P.h;
  const double sig0 = pl[3][dc] - n[AX] * (fwd ? h : 0.0);
  constexpr int O1 = AX == 0 ? 1 : 0, O2 = AX == 2 ? 1 : 2;
  const double sw = geo_swept_area(sig0, un, n[O1], n[O2], h, P.dt);
  return uf * sw / (h * h * P.dt);
}

// The face below cell (i, j, k) along AX (f its index along AX) from the
// values the caller loaded: the raw face velocity, alpha1 of the cell and of
// its neighbour below (the cell itself at f = 0), phi of both.  A donor in
// the band takes the full geo_face.
template <int AX, bool PHI>
__device__ __forceinline__ double geo_low_face(const DevParams& P, const double* __restrict__ a1,
                                               const double* const (&U)[3], const double* __restrict__ phi,
                                               const double* const (&pl)[4], int i, int j, int k, int f, double uraw,
                                               double ac, double alo, double pc, double plo) {
  double uf = uraw;   // as liquid_face_u
  if (PHI) {
    if (f > 0) uf = uraw - (pc - plo) / P.h;
    else if (pressure_dirichlet(P.kind[AX * 2])) uf = uraw - 2.0 * pc / P.h;
  }
  if (uf == 0.0) return 0.0;
  const bool fwd = uf > 0.0;
  if (fwd && f == 0) return 0.0;   // inflow through a box face
  const double ad = fwd ? alo : ac;
  if (ad > GEO_SURF_TOL && ad < 1.0 - GEO_SURF_TOL) return geo_face<AX>(P, a1, U, phi, pl, i, j, k);
  return uf * ad;
}

// PHI: the liquid is moved by u - G phi (phi given).  Every value the three
// faces below a cell need outside the band is loaded before any is used.
template <bool PHI>
__global__ void __launch_bounds__(BLOCK) k_geo_flux(DevParams P, const double* __restrict__ a1, const double* __restrict__ u,
                           const double* __restrict__ v, const double* __restrict__ w,
                           const double* __restrict__ phi, const double* __restrict__ pnx,
                           const double* __restrict__ pny, const double* __restrict__ pnz,
                           const double* __restrict__ ps, double* __restrict__ Fx, double* __restrict__ Fy,
                           double* __restrict__ Fz) {
  const double* const U[3] = {u, v, w};
  const double* const pl[4] = {pnx, pny, pnz, ps};
  const long long sx = (long long)P.ny * P.nz, sy = P.nz;
  const long long stride = (long long)gridDim.x * BLOCK;
  for (long long c = (long long)blockIdx.x * BLOCK + threadIdx.x; c < P.n; c += stride) {
    int i, j, k;
    decode(P, c, i, j, k);
    const long long ex = uidx(P, i, j, k), ey = vidx(P, i, j, k), ez = widx(P, i, j, k);
    const long long cx = i > 0 ? c - sx : c, cy = j > 0 ? c - sy : c, cz = k > 0 ? c - 1 : c;
    const double ux = u[ex], uy = v[ey], uz = w[ez];
    const double ac = a1[c], ax = a1[cx], ay = a1[cy], az = a1[cz];
    double pc = 0.0, px = 0.0, py = 0.0, pz = 0.0;
    if (PHI) {
      pc = phi[c];
      px = phi[cx];
      py = phi[cy];
      pz = phi[cz];
    }
    Fx[ex] = geo_low_face<0, PHI>(P, a1, U, phi, pl, i, j, k, i, ux, ac, ax, pc, px);
    Fy[ey] = geo_low_face<1, PHI>(P, a1, U, phi, pl, i, j, k, j, uy, ac, ay, pc, py);
    Fz[ez] = geo_low_face<2, PHI>(P, a1, U, phi, pl, i, j, k, k, uz, ac, az, pc, pz);
    if (i == P.nx - 1) Fx[uidx(P, P.nx, j, k)] = geo_face<0>(P, a1, U, phi, pl, P.nx, j, k);
    if (j == P.ny - 1) Fy[vidx(P, i, P.ny, k)] = geo_face<1>(P, a1, U, phi, pl, i, P.ny, k);
    if (k == P.nz - 1) Fz[widx(P, i, j, P.nz)] = geo_face<2>(P, a1, U, phi, pl, i, j, P.nz);
  }
}

}  // namespace

void launch_geo_fluxes(const DevParams& P, const double* a1, const double* u, const double* v, const double* w,
                       const double* phi, double* const (&planes)[4], double* Fx, double* Fy, double* Fz,
                       hipStream_t s) {
  k_plic<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a1, planes[0], planes[1], planes[2], planes[3]);
  if (phi)
    k_geo_flux<true><<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a1, u, v, w, phi, planes[0], planes[1], planes[2],
                                                        planes[3], Fx, Fy, Fz);
  else
    k_geo_flux<false><<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a1, u, v, w, nullptr, planes[0], planes[1], planes[2],
                                                         planes[3], Fx, Fy, Fz);
}

}  // namespace dsv
