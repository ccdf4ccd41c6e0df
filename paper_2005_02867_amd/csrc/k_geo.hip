// Geometric interface advection (advection = 1; Section 2.1, eq. 3): the
// liquid fluxes of the step from a plane per surface cell.
//   k_liquid_faces: the face velocities that move the liquid, u - G phi
//     (phi = 0 half a cell outside open faces) or u itself;
//   k_plic: per surface cell (tol < alpha1 < 1 - tol) the plane n.x = s,
//     n = -grad(alpha1)/|grad(alpha1)| by central differences (a ghost outside
//     the box repeats its neighbour), s leaving alpha1 h^3 of liquid;
//   k_geo_flux: per face, the liquid volume through it in the step divided by
//     h^2 dt: the face velocity times the time integral of the area the donor
//     (upwind) cell's plane submerges while it moves along n with the donor's
//     centre velocity; a donor without a plane gives U_f alpha1; inflow
//     through a box face carries no liquid.
// k_advect then takes these fluxes in place of its flux-limited liquid flux.
#include <hip/hip_runtime.h>

#include "ds_device.h"
#include "ds_geo.h"
#include "ds_kernels.h"
#include "ds_stencil.h"

namespace dsv {

namespace {

__global__ void __launch_bounds__(BLOCK) k_liquid_faces(DevParams P, const double* __restrict__ u, const double* __restrict__ v,
                               const double* __restrict__ w, const double* __restrict__ phi,
                               double* __restrict__ Ux, double* __restrict__ Uy, double* __restrict__ Uz) {
  const long long nu = (long long)(P.nx + 1) * P.ny * P.nz, nv = (long long)P.nx * (P.ny + 1) * P.nz;
  const long long nw = (long long)P.nx * P.ny * (P.nz + 1);
  long long b0, b1;
  block_range(nu + nv + nw, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    int i, j, k;
    if (e < nu) {
      decode3(e, P.ny, P.nz, i, j, k);
      Ux[e] = liquid_face_u(P, phi, u[e], (long long)j * P.nz + k, (long long)P.ny * P.nz, i, P.nx, 0);
    } else if (e < nu + nv) {
      const long long f = e - nu;
      decode3(f, P.ny + 1, P.nz, i, j, k);
      Uy[f] = liquid_face_u(P, phi, v[f], (long long)i * P.ny * P.nz + k, P.nz, j, P.ny, 1);
    } else {
      const long long f = e - nu - nv;
      decode3(f, P.ny, P.nz + 1, i, j, k);
      Uz[f] = liquid_face_u(P, phi, w[f], ((long long)i * P.ny + j) * P.nz, 1, k, P.nz, 2);
    }
  }
}

__global__ void __launch_bounds__(BLOCK) k_plic(DevParams P, const double* __restrict__ a1, double* __restrict__ pnx,
                       double* __restrict__ pny, double* __restrict__ pnz, double* __restrict__ ps) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double h = P.h;
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    const double a = a1[c];
    double n[3] = {0.0, 0.0, 0.0}, s = 0.0;
    if (a > GEO_SURF_TOL && a < 1.0 - GEO_SURF_TOL) {
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
    }
    pnx[c] = n[0];
    pny[c] = n[1];
    pnz[c] = n[2];
    ps[c] = s;
  }
}

// Liquid flux density (volume / (h^2 dt)) through face f of axis AX, the face
// between cells f-1 and f along AX at the other indices (o1, o2).
template <int AX>
__device__ __forceinline__ double geo_face(const DevParams& P, const double* __restrict__ a1,
                                           const double* const (&U)[3], const double* const (&pl)[4], int i, int j,
                                           int k) {
  const int fpos = AX == 0 ? i : (AX == 1 ? j : k);
  const int nax = AX == 0 ? P.nx : (AX == 1 ? P.ny : P.nz);
  const long long e = AX == 0 ? uidx(P, i, j, k) : (AX == 1 ? vidx(P, i, j, k) : widx(P, i, j, k));
  const double uf = U[AX][e];
  if (uf == 0.0) return 0.0;
  const bool fwd = uf > 0.0;
  if (fwd ? fpos == 0 : fpos == nax) return 0.0;   // inflow through a box face
  int d[3] = {i, j, k};
  if (fwd) d[AX] -= 1;
  const long long dc = cidx(P, d[0], d[1], d[2]);
  const double ad = a1[dc];
  const double n[3] = {pl[0][dc], pl[1][dc], pl[2][dc]};
  if (n[0] == 0.0 && n[1] == 0.0 && n[2] == 0.0) return uf * ad;
  // the donor's centre velocity and the plane's normal speed
  const double uc[3] = {0.5 * (U[0][uidx(P, d[0], d[1], d[2])] + U[0][uidx(P, d[0] + 1, d[1], d[2])]),
                        0.5 * (U[1][vidx(P, d[0], d[1], d[2])] + U[1][vidx(P, d[0], d[1] + 1, d[2])]),
                        0.5 * (U[2][widx(P, d[0], d[1], d[2])] + U[2][widx(P, d[0], d[1], d[2] + 1)])};
  const double un = uc[0] * n[0] + uc[1] * n[1] + uc[2] * n[2];
  const double h = P.h;
  const double sig0 = pl[3][dc] - n[AX] * (fwd ? h : 0.0);
  constexpr int O1 = AX == 0 ? 1 : 0, O2 = AX == 2 ? 1 : 2;
  const double sw = geo_swept_area(sig0, un, n[O1], n[O2], h, P.dt);
  return uf * sw / (h * h * P.dt);
}

__global__ void __launch_bounds__(BLOCK) k_geo_flux(DevParams P, const double* __restrict__ a1, const double* __restrict__ Ux,
                           const double* __restrict__ Uy, const double* __restrict__ Uz,
                           const double* __restrict__ pnx, const double* __restrict__ pny,
                           const double* __restrict__ pnz, const double* __restrict__ ps, double* __restrict__ Fx,
                           double* __restrict__ Fy, double* __restrict__ Fz) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double* const U[3] = {Ux, Uy, Uz};
  const double* const pl[4] = {pnx, pny, pnz, ps};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    Fx[uidx(P, i, j, k)] = geo_face<0>(P, a1, U, pl, i, j, k);
    Fy[vidx(P, i, j, k)] = geo_face<1>(P, a1, U, pl, i, j, k);
    Fz[widx(P, i, j, k)] = geo_face<2>(P, a1, U, pl, i, j, k);
    if (i == P.nx - 1) Fx[uidx(P, P.nx, j, k)] = geo_face<0>(P, a1, U, pl, P.nx, j, k);
    if (j == P.ny - 1) Fy[vidx(P, i, P.ny, k)] = geo_face<1>(P, a1, U, pl, i, P.ny, k);
    if (k == P.nz - 1) Fz[widx(P, i, j, P.nz)] = geo_face<2>(P, a1, U, pl, i, j, P.nz);
  }
}

}  // namespace

void launch_geo_fluxes(const DevParams& P, const double* a1, const double* u, const double* v, const double* w,
                       const double* phi, double* Ux, double* Uy, double* Uz, double* const (&planes)[4],
                       double* Fx, double* Fy, double* Fz, hipStream_t s) {
  const long long nf = (long long)(P.nx + 1) * P.ny * P.nz + (long long)P.nx * (P.ny + 1) * P.nz +
                       (long long)P.nx * P.ny * (P.nz + 1);
  k_liquid_faces<<<grid_blocks(nf), BLOCK, 0, s>>>(P, u, v, w, phi, Ux, Uy, Uz);
  k_plic<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a1, planes[0], planes[1], planes[2], planes[3]);
  k_geo_flux<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a1, Ux, Uy, Uz, planes[0], planes[1], planes[2], planes[3], Fx, Fy,
                                                Fz);
}

}  // namespace dsv
