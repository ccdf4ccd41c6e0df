// Step kernels of the VOF droplet-evaporation method (arXiv 2005.02867,
// Sections 2-3), FP64.  One thread per cell (or face), z fastest, each block
// streaming one contiguous range (XCD-aware order, see block_range).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ds_device.h"
#include "ds_kernels.h"
#include "ds_stencil.h"
#include "ds_thermo.h"

namespace dsv {

int grid_blocks(long long n) {
  long long nb = (n + BLOCK - 1) / BLOCK;
  if (nb > MAX_BLOCKS) nb = MAX_BLOCKS;
  nb = (nb + NXCD - 1) / NXCD * NXCD;
  return (int)nb;
}

// Tiles of the marching kernels: x chunks of at least 8 planes, as many as
// keep the tile count near MAX_BLOCKS; blocks walk the tiles grid-stride
// (a multiple of NXCD, at most MAX_BLOCKS, so per-block partials fit).
MarchGeom march_geom(const DevParams& P, int& blocks) {
  MarchGeom G;
  G.nzb = (P.nz + MZ - 1) / MZ;
  G.nyb = (P.ny + MY - 1) / MY;
  const long long yz = (long long)G.nzb * G.nyb;
  long long nxc = std::max(1LL, MAX_BLOCKS / yz);
  nxc = std::min(nxc, std::max(1LL, (long long)(P.nx + 7) / 8));
  G.xlen = (int)((P.nx + nxc - 1) / nxc);
  nxc = (P.nx + G.xlen - 1) / G.xlen;
  G.tiles = yz * nxc;
  long long nb = std::min<long long>(G.tiles, MAX_BLOCKS);
  nb = (nb + NXCD - 1) / NXCD * NXCD;
  blocks = (int)std::min<long long>(nb, MAX_BLOCKS);
  return G;
}

// ---------------------------------------------------------------- potential
// xi = xi0 (Df/2) / max(r, r_fib) at cell centres (eq. 29), centre x0.
__global__ void k_xi(DevParams P, double* xi) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    const double x = (i + 0.5) * P.h - P.x0[0], y = (j + 0.5) * P.h - P.x0[1], z = (k + 0.5) * P.h - P.x0[2];
    const double r = sqrt(x * x + y * y + z * z);
    xi[c] = P.xi0 * (0.5 * P.Df) / fmax(r, P.r_fib);
  }
}

// ---------------------------------------------------------------- S1-S3
// Interface cells (eps < alpha < 1-eps): central-difference gradient with a
// zero ghost outside the box, outward normal n = -grad/|grad|, march along n
// to the first gas cell (adj), evaporation flux at adj (eqs. 12-14) times
// |grad alpha| (eq. 17).  The march arithmetic is written with explicitly
// rounded operations so that each product and sum rounds on its own.
// Pass 1 (light, all cells): mraw = 0, adj = -2 off the interface; every
// interface cell (eps < alpha < 1 - eps) is appended, in cell order, to this
// block's list (wave ballots give each lane its slot), so pass 2 runs the
// march and the phase equilibrium only where they apply, one cell per lane.
// LIQ: list the liquid cells (alpha > eps_gas) instead and write nothing
// else (the literal species form's saturation pass).
template <bool LIQ>
__global__ void __launch_bounds__(BLOCK) k_interface_scan(DevParams P, const double* __restrict__ alpha,
                                                         double* __restrict__ mraw, int* __restrict__ adj,
                                                         int* __restrict__ band, int* __restrict__ band_count) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  __shared__ int wave_cnt[BLOCK / 64];
  __shared__ int base_sh;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  const long long cap = (long long)((P.n + gridDim.x - 1) / gridDim.x + BLOCK - 1) / BLOCK * BLOCK;
  int* list = band + (long long)blockIdx.x * cap;
  if (threadIdx.x == 0) base_sh = 0;
  __syncthreads();
  const long long span = b1 > b0 ? b1 - b0 : 0;
  for (long long off = 0; off < span; off += BLOCK) {
    const long long c = b0 + off + threadIdx.x;
    bool cand = false;
    if (c < b1) {
      const double a = alpha[c];
      if (LIQ) {
        cand = a > P.eps_gas;
      } else {
        cand = a > P.eps && a < 1.0 - P.eps;
        mraw[c] = 0.0;
        adj[c] = cand ? -1 : -2;
      }
    }
    const unsigned long long m = __ballot(cand);
    if (lane == 0) wave_cnt[wid] = __popcll(m);
    __syncthreads();
    int before = base_sh;
    for (int w = 0; w < wid; ++w) before += wave_cnt[w];
    if (cand) list[before + __popcll(m & ((1ull << lane) - 1ull))] = (int)c;
    __syncthreads();
    if (threadIdx.x == 0) {
      int tot = 0;
      for (int w = 0; w < BLOCK / 64; ++w) tot += wave_cnt[w];
      base_sh += tot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) band_count[blockIdx.x] = base_sh;
}

// Exclusive prefix sums of the per-block interface counts, in one workgroup:
// off[b] = sum of count[b'] over b' < b, off[nb] = the total (nb <= 2048).
__global__ void __launch_bounds__(1024) k_band_offsets(const int* __restrict__ count, int nb, int* __restrict__ off) {
  __shared__ int wsum[16];
  const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
  const int a = 2 * t < nb ? count[2 * t] : 0, b = 2 * t + 1 < nb ? count[2 * t + 1] : 0;
  int v = a + b;   // inclusive scan over the wave
  for (int o = 1; o < 64; o <<= 1) {
    const int y = __shfl_up(v, o, 64);
    if (lane >= o) v += y;
  }
  if (lane == 63) wsum[wid] = v;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wid; ++w) base += wsum[w];
  const int excl = base + v - (a + b);
  if (2 * t < nb) off[2 * t] = excl;
  if (2 * t + 1 < nb) off[2 * t + 1] = excl + a;
  if (t == 1023) off[nb] = base + v;
}

// Entry g of the per-block lists taken as one sequence: the list holding it
// is the largest b with off[b] <= g.
__device__ __forceinline__ long long band_entry(const int* __restrict__ band, const int* __restrict__ off, int nlists,
                                                long long cap, int g) {
  int lo = 0, hi = nlists - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  return band[(long long)lo * cap + (g - off[lo])];
}

// Pass 2 (interface cells, all lists taken as one sequence in cell order and
// dealt to full waves): central-difference gradient
// with a zero ghost outside the box, outward normal n = -grad/|grad|, march
// along n to the first gas cell (adj), evaporation flux at adj (eqs. 12-14)
// times |grad alpha| (eq. 17); the sums of eq. 20 and the interface count.
// The march arithmetic is written with explicitly rounded operations so that
// each product and sum rounds on its own.
__global__ void k_interface(DevParams P, const double* __restrict__ alpha, const double* __restrict__ T,
                            const double* __restrict__ omega, const double* __restrict__ u,
                            const double* __restrict__ v, const double* __restrict__ w,
                            const int* __restrict__ band, const int* __restrict__ off, int nlists, long long cap,
                            double* __restrict__ mraw, int* __restrict__ adj, double* partials,
                            unsigned* counter, double* scal) {
  double acc[3] = {0.0, 0.0, 0.0};
  const int total = off[nlists];
  for (int g = blockIdx.x * BLOCK + threadIdx.x; g < total; g += gridDim.x * BLOCK) {
    const long long c = band_entry(band, off, nlists, cap, g);
    const double a = alpha[c];
    double m = 0.0;
    int hit = -1;
    int i, j, k;
    decode(P, c, i, j, k);
    const double dx = __dsub_rn(alpha_or0(P, alpha, i + 1, j, k), alpha_or0(P, alpha, i - 1, j, k));
    const double dy = __dsub_rn(alpha_or0(P, alpha, i, j + 1, k), alpha_or0(P, alpha, i, j - 1, k));
    const double dz = __dsub_rn(alpha_or0(P, alpha, i, j, k + 1), alpha_or0(P, alpha, i, j, k - 1));
    const double nrm =
        __dsqrt_rn(__dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)));
    if (nrm > 0.0) {
      acc[2] += 1.0;
      const double nx = __ddiv_rn(-dx, nrm), ny = __ddiv_rn(-dy, nrm), nz = __ddiv_rn(-dz, nrm);
      const double bi = i + 0.5, bj = j + 0.5, bk = k + 0.5;
      int ti = 0, tj = 0, tk = 0;
      for (int s = 1; s <= P.smax; ++s) {
        const double sd = (double)s;
        ti = (int)floor(__dadd_rn(bi, __dmul_rn(sd, nx)));
        tj = (int)floor(__dadd_rn(bj, __dmul_rn(sd, ny)));
        tk = (int)floor(__dadd_rn(bk, __dmul_rn(sd, nz)));
        if (ti < 0 || tj < 0 || tk < 0 || ti >= P.nx || tj >= P.ny || tk >= P.nz) break;
        if (alpha[cidx(P, ti, tj, tk)] <= P.eps_gas) {
          hit = (int)cidx(P, ti, tj, tk);
          break;
        }
      }
      if (hit >= 0) {
        const double di = ti - i, dj = tj - j, dk = tk - k;
        const double d = P.h * sqrt(di * di + dj * dj + dk * dk);
        const double wa = omega[hit];
        const double va = 0.5 * (u[uidx(P, ti, tj, tk)] + u[uidx(P, ti + 1, tj, tk)]) * nx +
                          0.5 * (v[vidx(P, ti, tj, tk)] + v[vidx(P, ti, tj + 1, tk)]) * ny +
                          0.5 * (w[widx(P, ti, tj, tk)] + w[widx(P, ti, tj, tk + 1)]) * nz;
        double jd;
        if (P.species_form == 1) {
          // literal form: central grad(omega) at adj over the saturated liquid,
          // a ghost outside the box takes the adj value
          const double oxm = ti > 0 ? omega[hit - (long long)P.ny * P.nz] : wa;
          const double oxp = ti + 1 < P.nx ? omega[hit + (long long)P.ny * P.nz] : wa;
          const double oym = tj > 0 ? omega[hit - P.nz] : wa;
          const double oyp = tj + 1 < P.ny ? omega[hit + P.nz] : wa;
          const double ozm = tk > 0 ? omega[hit - 1] : wa;
          const double ozp = tk + 1 < P.nz ? omega[hit + 1] : wa;
          const double gx = (oxp - oxm) / (2.0 * P.h), gy = (oyp - oym) / (2.0 * P.h), gz = (ozp - ozm) / (2.0 * P.h);
          jd = -P.rho_G * P.D * (gx * nx + gy * ny + gz * nz);
        } else {
          const double wsat = mass_fraction(P, equilibrium_y(P, T[c]));
          jd = P.rho_G * P.D * (wsat - wa) / d;
        }
        const double jn = jd + P.rho_G * wa * va;
        m = jn * (nrm / (2.0 * P.h));
      }
    }
    const double f = sqrt(fmax(a * (1.0 - a), 0.0));
    acc[0] += m;
    acc[1] += f * m;
    mraw[c] = m;
    adj[c] = hit;
  }
  const int ops[3] = {RSUM, RSUM, RSUM};
  if (block_reduce_publish<3>(acc, ops, partials, counter)) {
    double tot[3];
    block_combine<3>(ops, partials, counter, tot);
    if (threadIdx.x == 0) {
      scal[SC_S1] = tot[0];
      scal[SC_S2] = tot[1];
      scal[SC_NINT] = tot[2];
      scal[SC_K] = tot[1] != 0.0 ? tot[0] / tot[1] : 0.0;
    }
  }
}

// Literal species form (Section 2.5, after eq. 23): every liquid cell
// (alpha > eps_gas, the complement of the march's gas test) takes the
// saturation value at its own temperature, omega = omega_sat(T) and
// c = rho_G theta omega; gas cells are left alone.  The liquid cells come
// from the lists of k_interface_scan<true> (a light pass over all cells at
// full occupancy) and are dealt to full waves, so the per-cell equilibrium
// solves, whose code holds 128 VGPRs, run side by side on every compute
// unit and no wave of this kernel streams gas cells.
__global__ void k_liquid_saturation(DevParams P, const double* __restrict__ alpha, const double* __restrict__ T,
                                    const int* __restrict__ band, const int* __restrict__ off, int nlists,
                                    long long cap, double* __restrict__ omega, double* __restrict__ c) {
  const int total = off[nlists];
  for (int g = blockIdx.x * BLOCK + threadIdx.x; g < total; g += gridDim.x * BLOCK) {
    const long long e = band_entry(band, off, nlists, cap, g);
    const double a = alpha[e];
    const double ws = mass_fraction(P, equilibrium_y(P, T[e]));
    const double th = fmax(1.0 - clamp01(a), P.theta_min);
    omega[e] = ws;
    c[e] = P.rho_G * th * ws;
  }
}

// ---------------------------------------------------------------- S4 + eq. 4
// mdot = K f(alpha) mdot_raw (eqs. 19-21), alpha1 = alpha - dt mdot / rho_L.
__global__ void k_source(DevParams P, const double* __restrict__ alpha, const double* __restrict__ mraw,
                         const double* __restrict__ scal, double* __restrict__ mdot,
                         double* __restrict__ a1) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double K = scal[SC_K];
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    const double a = alpha[c];
    const double f = sqrt(fmax(a * (1.0 - a), 0.0));
    const double m = K * f * mraw[c];
    mdot[c] = m;
    a1[c] = a - P.dt * m / P.rho_L;
  }
}

// ---------------------------------------------------------------- S5
// Fluxes and update of one cell from its line values: A, O, TT hold alpha1,
// omega and T at offsets -2, -1, +1, +2 along each axis (index 0..3), h whether
// those cells exist; PH phi at -1, +1; uf the six face velocities.  The faces
// are formed with selects (no load waits on the upwind side).
__device__ __forceinline__ void advect_cell(const DevParams& P, const int (&pos)[3], const double (&uf)[3][2],
                                            double A0, double O0, double T0, double P0, const double (&A)[3][4],
                                            const double (&O)[3][4], const double (&TT)[3][4],
                                            const double (&PH)[3][2], const bool (&h)[3][4], bool has_phi,
                                            double cv, double (&acc)[2], double& an, double& cn, double& tn) {
  const int nn[3] = {P.nx, P.ny, P.nz};
  const double ih = 1.0 / P.h;
  double da = 0.0, dc = 0.0, dT = 0.0;
#pragma unroll
  for (int ax = 0; ax < 3; ++ax) {
    const int q = pos[ax], n = nn[ax];
    const bool lo_in = q > 0, hi_in = q < n - 1;
    double F[2], G[2], H[2];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const double ufv = uf[ax][sd];
      const bool in = sd == 0 ? lo_in : hi_in;
      // interior face: (m, a, b, p) = (-2, -1, 0, +1) below the cell, (-1, 0, +1, +2) above
      auto face = [&](const double (&L)[4], double c0, double vel) {
        return sd == 0 ? tvd_face(L[0], L[1], c0, L[2], h[ax][0], h[ax][2], vel)
                       : tvd_face(L[1], c0, L[2], L[3], h[ax][1], h[ax][3], vel);
      };
      const double af = in ? face(A[ax], A0, ufv) : box_face(A0, 0.0, ufv, sd);
      const double of = in ? face(O[ax], O0, ufv) : box_face(O0, 0.0, ufv, sd);
      if (has_phi) {
        double ul;
        if (sd == 0)
          ul = in ? ufv - (P0 - PH[ax][0]) * ih
                  : (pressure_dirichlet(P.kind[ax * 2]) ? ufv - 2.0 * P0 * ih : ufv);
        else
          ul = in ? ufv - (PH[ax][1] - P0) * ih
                  : (pressure_dirichlet(P.kind[ax * 2 + 1]) ? ufv + 2.0 * P0 * ih : ufv);
        F[sd] = ul * (in ? face(A[ax], A0, ul) : box_face(A0, 0.0, ul, sd));
      } else {
        F[sd] = ufv * af;
      }
      G[sd] = P.rho_G * of * (1.0 - af) * ufv;
      if (P.solve_energy) {
        const double Tf = in ? face(TT[ax], T0, ufv) : box_face(T0, P.T_amb, ufv, sd);
        H[sd] = ufv * (Tf - T0);
      } else {
        H[sd] = 0.0;
      }
    }
    da += F[1] - F[0];
    dc += G[1] - G[0];
    dT += H[1] - H[0];
    if (!lo_in) {
      acc[0] -= F[0];
      acc[1] -= G[0];
    }
    if (!hi_in) {
      acc[0] += F[1];
      acc[1] += G[1];
    }
  }
  const double s = P.dt / P.h;
  an = A0 - s * da;
  cn = cv - s * dc;
  tn = P.solve_energy ? T0 - s * dT : T0;
}

__device__ __forceinline__ void advect_publish(const DevParams& P, double (&acc)[2], double* partials,
                                               unsigned* counter, double* scal) {
  const int ops[2] = {RSUM, RSUM};
  if (block_reduce_publish<2>(acc, ops, partials, counter)) {
    double tot[2];
    block_combine<2>(ops, partials, counter, tot);
    if (threadIdx.x == 0) {
      const double area_dt = P.h * P.h * P.dt;
      scal[SC_BL] = P.rho_L * area_dt * tot[0];
      scal[SC_BV_ADV] = area_dt * tot[1];
    }
  }
}

// ---------------------------------------------------------------- marching tiles
// The explicit stencil kernels march along x over tiles of MZ = 64 z (one
// wavefront per row) by MY = 4 y rows.  Each x-plane of a tile is staged in
// LDS once with its y/z halo, three planes in flight: the loads of plane x+3
// are issued before plane x is computed and land in plane x's slot after it,
// so one barrier per plane separates every slot's reads from its next
// writes.  The x neighbours of a thread's own column ride along in registers.

// Tile of a block's logical number t (z tiles fastest, then y, then x chunks).
__device__ __forceinline__ void march_tile(const MarchGeom& G, long long t, int& x0, int& y0, int& z0) {
  const long long q = t / G.nzb;
  z0 = (int)(t - q * G.nzb) * MZ;
  y0 = (int)(q % G.nyb) * MY;
  x0 = (int)(q / G.nyb) * G.xlen;
}
// Logical block number: the blocks one XCD receives (round-robin dealing)
// take consecutive numbers, so neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int march_logical() {
  const int per = gridDim.x / NXCD;
  return (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
}

// Advection tiles: alpha1, omega, T with a halo of 2 (68 x 8), phi with 1
// (66 x 6).  The halo ring of a tile (the entries outside the 64 x 4 centre)
// is enumerated as: H full rows on top, H full rows at the bottom, then the
// H columns at either end of the middle rows.
constexpr int AHZ = MZ + 4, AHY = MY + 4, ATILE = AHZ * AHY, ARING = ATILE - MZ * MY;
constexpr int PHZ = MZ + 2, PHY = MY + 2, PTILE = PHZ * PHY, PRING = PTILE - MZ * MY;

template <int H>
__device__ __forceinline__ void ring_entry(int e, int& r, int& c) {
  constexpr int TZ = MZ + 2 * H, top = H * TZ;
  if (e < top) {
    r = e / TZ;
    c = e - r * TZ;
  } else if (e < 2 * top) {
    e -= top;
    const int q = e / TZ;
    r = MY + H + q;
    c = e - q * TZ;
  } else {
    e -= 2 * top;
    const int q = e / (2 * H), s = e - q * (2 * H);
    r = H + q;
    c = s < H ? s : MZ + s;
  }
}

// One x-plane of the advection tile in registers: the thread's own centre
// value of each field, then its share of the halo rings.
struct AdvPlane {
  double cA, cO, cT, cP;
  double rA[2], rO[2], rT[2], rP;
};

__device__ __forceinline__ void adv_fetch(const DevParams& P, const double* __restrict__ a1,
                                          const double* __restrict__ omega, const double* __restrict__ T,
                                          const double* __restrict__ phi, int X, int xcen, int xhalo, int y0,
                                          int z0, bool live, long long col, AdvPlane& f) {
  const long long plane = (long long)P.ny * P.nz;
  const bool cin = live && X >= 0 && X < xcen;
  const long long cg = cin ? X * plane + col : 0;
  f.cA = cin ? a1[cg] : 0.0;
  f.cO = cin ? omega[cg] : 0.0;
  f.cT = cin ? T[cg] : 0.0;
  f.cP = (cin && phi) ? phi[cg] : 0.0;
  const bool hin = X >= 0 && X < xhalo;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    int r = 0, c = 0;
    if (e < ARING) ring_entry<2>(e, r, c);
    const int gj = y0 - 2 + r, gk = z0 - 2 + c;
    const bool in = hin && e < ARING && gj >= 0 && gj < P.ny && gk >= 0 && gk < P.nz;
    const long long g = in ? X * plane + (long long)gj * P.nz + gk : 0;
    f.rA[q] = in ? a1[g] : 0.0;
    f.rO[q] = in ? omega[g] : 0.0;
    f.rT[q] = in ? T[g] : 0.0;
  }
  {
    const int e = threadIdx.x;
    int r = 0, c = 0;
    if (e < PRING) ring_entry<1>(e, r, c);
    const int gj = y0 - 1 + r, gk = z0 - 1 + c;
    const bool in = phi && hin && e < PRING && gj >= 0 && gj < P.ny && gk >= 0 && gk < P.nz;
    f.rP = in ? phi[X * plane + (long long)gj * P.nz + gk] : 0.0;
  }
}

__device__ __forceinline__ void adv_store(const AdvPlane& f, double (*sF)[ATILE], double* sP, int ty, int tz) {
  const int ce = (ty + 2) * AHZ + tz + 2;
  sF[0][ce] = f.cA;
  sF[1][ce] = f.cO;
  sF[2][ce] = f.cT;
  sP[(ty + 1) * PHZ + tz + 1] = f.cP;
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    if (e < ARING) {
      int r, c;
      ring_entry<2>(e, r, c);
      sF[0][r * AHZ + c] = f.rA[q];
      sF[1][r * AHZ + c] = f.rO[q];
      sF[2][r * AHZ + c] = f.rT[q];
    }
  }
  if (threadIdx.x < PRING) {
    int r, c;
    ring_entry<1>(threadIdx.x, r, c);
    sP[r * PHZ + c] = f.rP;
  }
}

// Face velocities and c of the thread's cell in plane X.
struct AdvFaces {
  double u0, u1, v0, v1, w0, w1, c;
};
__device__ __forceinline__ void adv_faces(const DevParams& P, const double* __restrict__ u,
                                          const double* __restrict__ v, const double* __restrict__ w,
                                          const double* __restrict__ c, int X, int x1, int j, int k, bool live,
                                          AdvFaces& F) {
  const bool in = live && X < x1;
  const int i = in ? X : 0, jj = in ? j : 0, kk = in ? k : 0;
  F.u0 = in ? u[uidx(P, i, jj, kk)] : 0.0;
  F.u1 = in ? u[uidx(P, i + 1, jj, kk)] : 0.0;
  F.v0 = in ? v[vidx(P, i, jj, kk)] : 0.0;
  F.v1 = in ? v[vidx(P, i, jj + 1, kk)] : 0.0;
  F.w0 = in ? w[widx(P, i, jj, kk)] : 0.0;
  F.w1 = in ? w[widx(P, i, jj, kk + 1)] : 0.0;
  F.c = in ? c[cidx(P, i, jj, kk)] : 0.0;
}

// Advection of alpha1, c and T (eq. 3 with the liquid-transport velocity,
// the vapour flux and the temperature transport), marching along x.
__global__ void __launch_bounds__(BLOCK)
k_advect(DevParams P, MarchGeom G, const double* __restrict__ a1, const double* __restrict__ omega,
         const double* __restrict__ T, const double* __restrict__ c, const double* __restrict__ u,
         const double* __restrict__ v, const double* __restrict__ w, const double* __restrict__ phi,
         double* __restrict__ a_new, double* __restrict__ c_new, double* __restrict__ T_new, double* partials,
         unsigned* counter, double* scal) {
  __shared__ double sF[3][3][ATILE];   // slot (x mod 3), field (alpha1, omega, T)
  __shared__ double sP[3][PTILE];      // slot, phi
  const int tz = threadIdx.x % MZ, ty = threadIdx.x / MZ;
  double acc[2] = {0.0, 0.0};   // outward liquid volume flux, vapour mass flux (per area)
  const long long plane = (long long)P.ny * P.nz;
  for (long long t = march_logical(); t < G.tiles; t += gridDim.x) {
    int x0, y0, z0;
    march_tile(G, t, x0, y0, z0);
    const int x1 = min(x0 + G.xlen, P.nx);
    const int xcen = min(P.nx, x1 + 2);   // own columns are read up to x1 + 1, halos up to x1 - 1
    const int j = y0 + ty, k = z0 + tz;
    const bool live = j < P.ny && k < P.nz;
    const long long col = live ? (long long)j * P.nz + k : 0;
    // x window of the own column: planes x-2 .. x+2 (phi: x-1 .. x+1 used)
    double wA[5], wO[5], wT[5], wP[5];
    __syncthreads();   // the previous tile's last reads of the slots
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const int X = x0 - 2 + q;
      const bool in = live && X >= 0;
      const long long g = in ? X * plane + col : 0;
      wA[q] = in ? a1[g] : 0.0;
      wO[q] = in ? omega[g] : 0.0;
      wT[q] = in ? T[g] : 0.0;
      wP[q] = (in && phi) ? phi[g] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      AdvPlane f;
      adv_fetch(P, a1, omega, T, phi, x0 + q, xcen, x1, y0, z0, live, col, f);
      adv_store(f, sF[(x0 + q) % 3], sP[(x0 + q) % 3], ty, tz);
      wA[2 + q] = f.cA;
      wO[2 + q] = f.cO;
      wT[2 + q] = f.cT;
      wP[2 + q] = f.cP;
    }
    AdvFaces F;
    adv_faces(P, u, v, w, c, x0, x1, j, k, live, F);
    __syncthreads();
    int slot = x0 % 3;
    for (int x = x0; x < x1; ++x) {
      AdvPlane nf;
      adv_fetch(P, a1, omega, T, phi, x + 3, xcen, x1, y0, z0, live, col, nf);
      AdvFaces NF;
      adv_faces(P, u, v, w, c, x + 1, x1, j, k, live, NF);
      if (live) {
        const double(*S)[ATILE] = sF[slot];
        const double* SP = sP[slot];
        const int pos[3] = {x, j, k};
        const double uf[3][2] = {{F.u0, F.u1}, {F.v0, F.v1}, {F.w0, F.w1}};
        const int ce = (ty + 2) * AHZ + tz + 2;
        double A[3][4], O[3][4], TT[3][4], PH[3][2];
        const double* fs[3] = {wA, wO, wT};
        double(*dst[3])[4] = {A, O, TT};
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const double* wf = fs[f];
          dst[f][0][0] = wf[0];
          dst[f][0][1] = wf[1];
          dst[f][0][2] = wf[3];
          dst[f][0][3] = wf[4];
          dst[f][1][0] = S[f][ce - 2 * AHZ];
          dst[f][1][1] = S[f][ce - AHZ];
          dst[f][1][2] = S[f][ce + AHZ];
          dst[f][1][3] = S[f][ce + 2 * AHZ];
          dst[f][2][0] = S[f][ce - 2];
          dst[f][2][1] = S[f][ce - 1];
          dst[f][2][2] = S[f][ce + 1];
          dst[f][2][3] = S[f][ce + 2];
        }
        const int pe = (ty + 1) * PHZ + tz + 1;
        PH[0][0] = wP[1];
        PH[0][1] = wP[3];
        PH[1][0] = SP[pe - PHZ];
        PH[1][1] = SP[pe + PHZ];
        PH[2][0] = SP[pe - 1];
        PH[2][1] = SP[pe + 1];
        bool h[3][4];
        const int nn[3] = {P.nx, P.ny, P.nz};
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          const int q = pos[ax], n = nn[ax];
          h[ax][0] = q >= 2;
          h[ax][1] = q >= 1;
          h[ax][2] = q + 1 <= n - 1;
          h[ax][3] = q + 2 <= n - 1;
        }
        double an, cn, tn;
        advect_cell(P, pos, uf, wA[2], wO[2], wT[2], wP[2], A, O, TT, PH, h, phi != nullptr, F.c, acc, an, cn,
                    tn);
        const long long cc = x * plane + col;
        a_new[cc] = an;
        c_new[cc] = cn;
        T_new[cc] = tn;
      }
      __syncthreads();   // every read of this slot is done
      adv_store(nf, sF[slot], sP[slot], ty, tz);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        wA[q] = wA[q + 1];
        wO[q] = wO[q + 1];
        wT[q] = wT[q + 1];
        wP[q] = wP[q + 1];
      }
      wA[4] = nf.cA;
      wO[4] = nf.cO;
      wT[4] = nf.cT;
      wP[4] = nf.cP;
      F = NF;
      slot = slot == 2 ? 0 : slot + 1;
    }
  }
  advect_publish(P, acc, partials, counter, scal);
}

// ---------------------------------------------------------------- S6-S8
// Energy, eq. 8 after the advection: (rho cp/dt) T - div(k grad T) = (rho cp/dt) T' - mdot dh.
__global__ void k_energy_setup(DevParams P, const double* __restrict__ a_new, const double* __restrict__ Tp,
                               const double* __restrict__ mdot, const double* __restrict__ u,
                               const double* __restrict__ v, const double* __restrict__ w,
                               double* __restrict__ qc, double* __restrict__ diag, double* __restrict__ b,
                               F32Out fo) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double ih2 = 1.0 / (P.h * P.h);
  const double Kb = 2.0 * P.k_G * ih2;
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    double an[6];
    bool has[6];
    nbr6(P, a_new, c, i, j, k, an, has);
    const double ab = clamp01(a_new[c]);
    const double rho = mix(ab, P.rho_L, P.rho_G), cp = mix(ab, P.cp_L, P.cp_G), kc = mix(ab, P.k_L, P.k_G);
    const double m = rho * cp / P.dt;
    double d = m, rhs = m * Tp[c] - mdot[c] * P.dh;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        if (has[ax * 2 + sd]) {
          const double kn = mix(clamp01(an[ax * 2 + sd]), P.k_L, P.k_G);
          d += ih2 * 0.5 * (kc + kn);
        } else if (scalar_dirichlet(P.kind[ax * 2 + sd], bface_u(P, u, v, w, ax, sd, i, j, k), sd)) {
          d += Kb;
          rhs += Kb * P.T_amb;
        }
      }
    qc[c] = kc;
    diag[c] = d;
    b[c] = rhs;
    if (fo.q) {
      fo.q[c] = (float)kc;
      fo.d[c] = (float)d;
    }
  }
}

// Species, eq. 9 for c = rho_G theta omega: (rho_G theta/dt) w - div(rho_G D theta grad w) = c'/dt + mdot
// (without mdot in the literal species form).
__global__ void k_species_setup(DevParams P, const double* __restrict__ a_new, const double* __restrict__ cp_,
                                const double* __restrict__ mdot, const double* __restrict__ u,
                                const double* __restrict__ v, const double* __restrict__ w,
                                double* __restrict__ qc, double* __restrict__ diag, double* __restrict__ b,
                                double* __restrict__ om0, F32Out fo) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double sc = P.rho_G * P.D / (P.h * P.h);
  const double Kb = 2.0 * sc;
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    double an[6];
    bool has[6];
    nbr6(P, a_new, c, i, j, k, an, has);
    const double th = fmax(1.0 - clamp01(a_new[c]), P.theta_min);
    double d = P.rho_G * th / P.dt;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        if (has[ax * 2 + sd]) {
          const double tn = fmax(1.0 - clamp01(an[ax * 2 + sd]), P.theta_min);
          d += sc * 0.5 * (th + tn);
        } else if (scalar_dirichlet(P.kind[ax * 2 + sd], bface_u(P, u, v, w, ax, sd, i, j, k), sd)) {
          d += Kb;
        }
      }
    qc[c] = th;
    diag[c] = d;
    // the literal species form has no mdot source (the saturated liquid feeds the gas)
    b[c] = P.species_form == 1 ? cp_[c] / P.dt : cp_[c] / P.dt + mdot[c];
    if (om0) om0[c] = cp_[c] / (P.rho_G * th);
    if (fo.q) {
      fo.q[c] = (float)th;
      fo.d[c] = (float)d;
    }
  }
}

// Flux-form vapour update after the implicit solve; diffusive boundary outflow tally.
__global__ void k_species_update(DevParams P, const double* __restrict__ a_new, const double* __restrict__ cp_,
                                 const double* __restrict__ mdot, const double* __restrict__ om,
                                 const double* __restrict__ u, const double* __restrict__ v,
                                 const double* __restrict__ w, double* __restrict__ cout,
                                 double* __restrict__ omega, double* partials, unsigned* counter,
                                 double* scal) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double sc = P.rho_G * P.D / (P.h * P.h);
  const double Kb = 2.0 * sc;
  double acc[1] = {0.0};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    double an[6], on[6];
    bool has[6];
    nbr6(P, a_new, c, i, j, k, an, has);
    nbr6(P, om, c, i, j, k, on, has);
    const double th = fmax(1.0 - clamp01(a_new[c]), P.theta_min);
    const double oc = om[c];
    double face = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        if (has[ax * 2 + sd]) {
          const double tn = fmax(1.0 - clamp01(an[ax * 2 + sd]), P.theta_min);
          face += sc * 0.5 * (th + tn) * (oc - on[ax * 2 + sd]);
        } else if (scalar_dirichlet(P.kind[ax * 2 + sd], bface_u(P, u, v, w, ax, sd, i, j, k), sd)) {
          face += Kb * oc;
          acc[0] += Kb * oc;
        }
      }
    const double cn = (P.species_form == 1 ? cp_[c] : cp_[c] + P.dt * mdot[c]) - P.dt * face;
    cout[c] = cn;
    omega[c] = cn / (P.rho_G * th);
  }
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double tot[1];
    block_combine<1>(ops, partials, counter, tot);
    if (threadIdx.x == 0) scal[SC_BV_DIFF] = P.dt * P.h * P.h * P.h * tot[0];
  }
}

// ---------------------------------------------------------------- S9
// Predictor on an interior face normal to AX (eq. 30 / rho, mu = 0):
// first-order upwind advection along AX (face neighbours bn, fn), transverse
// advection along the two other axes (ascending) with the four-point
// averaged velocity vb and the one-sided differences to lo / hi (zero-
// gradient ghosts already substituted), gravity on the density jump and the
// potential force on the xi jump between the cells L and R either side.
// (i, j, k): the face's indices in its face array.
template <int AX>
__device__ __forceinline__ double predictor_interior(const DevParams& P, double uc, double bn, double fn,
                                                     const double (&vb)[2], const double (&lo)[2],
                                                     const double (&hi)[2], double aL_, double aR_, double xiL,
                                                     double xiR, int i, int j, int k, double ih) {
  const double back = (uc - bn) * ih, fwd = (fn - uc) * ih;
  double adv = uc * (uc > 0.0 ? back : fwd);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double d = (vb[q] > 0.0 ? uc - lo[q] : hi[q] - uc) * ih;
    adv += vb[q] * d;
  }
  const double aL = clamp01(aL_), aR = clamp01(aR_);
  const double rL = mix(aL, P.rho_L, P.rho_G), rR = mix(aR, P.rho_L, P.rho_G);
  const double bf = 0.5 * (1.0 / rL + 1.0 / rR);
  const double xf = (AX == 0 ? i : i + 0.5) * P.h - P.x0[0];
  const double yf = (AX == 1 ? j : j + 0.5) * P.h - P.x0[1];
  const double zf = (AX == 2 ? k : k + 0.5) * P.h - P.x0[2];
  const double gr = P.g[0] * xf + P.g[1] * yf + P.g[2] * zf;
  const double force = -gr * (rR - rL) * ih * bf + 0.5 * (aL + aR) * (xiR - xiL) * ih;
  return uc - P.dt * adv + P.dt * force;
}
// Box face (side 0: low, 1: high) normal to AX: walls hold 0, the inlet w_in,
// open and far-field faces keep u^n.
__device__ __forceinline__ double predictor_box(const DevParams& P, int ax, int side, double uc) {
  const int kind = P.kind[ax * 2 + side];
  return kind == WALL ? 0.0 : (kind == INLET ? P.w_in : uc);
}

// Predictor tiles: u, v, w, alpha and xi planes with a halo of 1 (66 x 6,
// rows y0-1 .. y0+4, columns z0-1 .. z0+64); v and w keep their extra face
// row / column in it.
constexpr int QZ = MZ + 2, QY = MY + 2, QTILE = QZ * QY;
constexpr int QF = 5;   // u, v, w, alpha, xi

struct PredPlane {
  double e[QF][2];
};
// Plane X of every field, entries threadIdx.x and threadIdx.x + BLOCK of the
// tile (row-major); X up to xmax (u has nx + 1 planes, the others nx).
__device__ __forceinline__ void pred_fetch(const DevParams& P, const double* __restrict__ u,
                                           const double* __restrict__ v, const double* __restrict__ w,
                                           const double* __restrict__ a, const double* __restrict__ xi, int X,
                                           int xmax, int y0, int z0, PredPlane& f) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    const int r = e / QZ, c = e - r * QZ;
    const int gj = y0 - 1 + r, gk = z0 - 1 + c;
    const bool ok = e < QTILE && X >= 0 && X <= xmax && gj >= 0 && gk >= 0;
    const bool cell = ok && X < P.nx && gj < P.ny && gk < P.nz;
    const bool uin = ok && gj < P.ny && gk < P.nz;                  // X <= nx
    const bool vin = ok && X < P.nx && gj <= P.ny && gk < P.nz;
    const bool win = ok && X < P.nx && gj < P.ny && gk <= P.nz;
    f.e[0][q] = uin ? u[uidx(P, X, gj, gk)] : 0.0;
    f.e[1][q] = vin ? v[vidx(P, X, gj, gk)] : 0.0;
    f.e[2][q] = win ? w[widx(P, X, gj, gk)] : 0.0;
    f.e[3][q] = cell ? a[cidx(P, X, gj, gk)] : 0.0;
    f.e[4][q] = cell ? xi[cidx(P, X, gj, gk)] : 0.0;
  }
}
__device__ __forceinline__ void pred_store(const PredPlane& f, double (*S)[QTILE]) {
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    if (e < QTILE) {
#pragma unroll
      for (int fl = 0; fl < QF; ++fl) S[fl][e] = f.e[fl][q];
    }
  }
}

// u*, v*, w* of every face, marching along x: the thread of cell (x, j, k)
// writes the faces (x, j, k) of the three arrays and, on the high box faces,
// the face beyond.  Plane x and x+1 tiles give the y/z neighbours and the
// x+1 values; the x-1 values are kept from the previous plane.
__global__ void __launch_bounds__(BLOCK)
k_predictor(DevParams P, MarchGeom G, const double* __restrict__ a_new, const double* __restrict__ xi,
            const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
            double* __restrict__ us, double* __restrict__ vs, double* __restrict__ ws) {
  __shared__ double sQ[3][QF][QTILE];   // slot (x mod 3), field
  const int tz = threadIdx.x % MZ, ty = threadIdx.x / MZ;
  const double ih = 1.0 / P.h;
  constexpr int FU = 0, FV = 1, FW = 2, FA = 3, FX = 4;
  for (long long t = march_logical(); t < G.tiles; t += gridDim.x) {
    int x0, y0, z0;
    march_tile(G, t, x0, y0, z0);
    const int x1 = min(x0 + G.xlen, P.nx);
    const int j = y0 + ty, k = z0 + tz;
    const bool live = j < P.ny && k < P.nz;
    // plane x-1 values of the own column: u, v (j, j+1), w (k, k+1), alpha, xi
    double pu, pv0, pv1, pw0, pw1, pa, px;
    {
      const bool in = live && x0 >= 1;
      const int X = in ? x0 - 1 : 0, jj = in ? j : 0, kk = in ? k : 0;
      pu = in ? u[uidx(P, X, jj, kk)] : 0.0;
      pv0 = in ? v[vidx(P, X, jj, kk)] : 0.0;
      pv1 = in ? v[vidx(P, X, jj + 1, kk)] : 0.0;
      pw0 = in ? w[widx(P, X, jj, kk)] : 0.0;
      pw1 = in ? w[widx(P, X, jj, kk + 1)] : 0.0;
      pa = in ? a_new[cidx(P, X, jj, kk)] : 0.0;
      px = in ? xi[cidx(P, X, jj, kk)] : 0.0;
    }
    __syncthreads();   // the previous tile's last reads of the slots
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      PredPlane f;
      pred_fetch(P, u, v, w, a_new, xi, x0 + q, x1, y0, z0, f);
      pred_store(f, sQ[(x0 + q) % 3]);
    }
    __syncthreads();
    int slot = x0 % 3;
    for (int x = x0; x < x1; ++x) {
      PredPlane nf;
      pred_fetch(P, u, v, w, a_new, xi, x + 3, x1, y0, z0, nf);
      const int s1 = slot == 2 ? 0 : slot + 1;
      if (live) {
        const int ce = (ty + 1) * QZ + tz + 1;
        auto T0 = [&](int f, int dy, int dz) { return sQ[slot][f][ce + dy * QZ + dz]; };
        auto T1 = [&](int f, int dy, int dz) { return sQ[s1][f][ce + dy * QZ + dz]; };
        const double uc = T0(FU, 0, 0), vc = T0(FV, 0, 0), wc = T0(FW, 0, 0);
        const double ac = T0(FA, 0, 0), xc = T0(FX, 0, 0);
        const double un = T1(FU, 0, 0);   // u(x+1, j, k)
        double ru, rv, rw;
        // u face (x, j, k)
        if (x == 0) {
          ru = predictor_box(P, 0, 0, uc);
        } else {
          const double vb[2] = {0.25 * (pv0 + pv1 + vc + T0(FV, 1, 0)), 0.25 * (pw0 + pw1 + wc + T0(FW, 0, 1))};
          const double lo[2] = {j >= 1 ? T0(FU, -1, 0) : uc, k >= 1 ? T0(FU, 0, -1) : uc};
          const double hi[2] = {j <= P.ny - 2 ? T0(FU, 1, 0) : uc, k <= P.nz - 2 ? T0(FU, 0, 1) : uc};
          ru = predictor_interior<0>(P, uc, pu, un, vb, lo, hi, pa, ac, px, xc, x, j, k, ih);
        }
        // v face (x, j, k)
        if (j == 0) {
          rv = predictor_box(P, 1, 0, vc);
        } else {
          const double vb[2] = {0.25 * (T0(FU, -1, 0) + T1(FU, -1, 0) + uc + un),
                                0.25 * (T0(FW, -1, 0) + T0(FW, -1, 1) + wc + T0(FW, 0, 1))};
          const double lo[2] = {x >= 1 ? pv0 : vc, k >= 1 ? T0(FV, 0, -1) : vc};
          const double hi[2] = {x <= P.nx - 2 ? T1(FV, 0, 0) : vc, k <= P.nz - 2 ? T0(FV, 0, 1) : vc};
          rv = predictor_interior<1>(P, vc, T0(FV, -1, 0), T0(FV, 1, 0), vb, lo, hi, T0(FA, -1, 0), ac,
                                     T0(FX, -1, 0), xc, x, j, k, ih);
        }
        // w face (x, j, k)
        if (k == 0) {
          rw = predictor_box(P, 2, 0, wc);
        } else {
          const double vb[2] = {0.25 * (T0(FU, 0, -1) + T1(FU, 0, -1) + uc + un),
                                0.25 * (T0(FV, 0, -1) + T0(FV, 1, -1) + vc + T0(FV, 1, 0))};
          const double lo[2] = {x >= 1 ? pw0 : wc, j >= 1 ? T0(FW, -1, 0) : wc};
          const double hi[2] = {x <= P.nx - 2 ? T1(FW, 0, 0) : wc, j <= P.ny - 2 ? T0(FW, 1, 0) : wc};
          rw = predictor_interior<2>(P, wc, T0(FW, 0, -1), T0(FW, 0, 1), vb, lo, hi, T0(FA, 0, -1), ac,
                                     T0(FX, 0, -1), xc, x, j, k, ih);
        }
        us[uidx(P, x, j, k)] = ru;
        vs[vidx(P, x, j, k)] = rv;
        ws[widx(P, x, j, k)] = rw;
        if (x == P.nx - 1) us[uidx(P, P.nx, j, k)] = predictor_box(P, 0, 1, un);
        if (j == P.ny - 1) vs[vidx(P, x, P.ny, k)] = predictor_box(P, 1, 1, T0(FV, 1, 0));
        if (k == P.nz - 1) ws[widx(P, x, j, P.nz)] = predictor_box(P, 2, 1, T0(FW, 0, 1));
        pu = uc;
        pv0 = vc;
        pv1 = T0(FV, 1, 0);
        pw0 = wc;
        pw1 = T0(FW, 0, 1);
        pa = ac;
        px = xc;
      }
      __syncthreads();   // every read of this slot is done
      pred_store(nf, sQ[slot]);
      slot = s1;
    }
  }
}

// ---------------------------------------------------------------- S10 setup
// Pressure: sum_f (dt/h^2) (1/rho)_f (p_c - p_nb) = mdot (1/rho_G - 1/rho_L) - div u*.
__global__ void k_pressure_setup(DevParams P, const double* __restrict__ a_new, const double* __restrict__ mdot,
                                 const double* __restrict__ us, const double* __restrict__ vs,
                                 const double* __restrict__ ws, double* __restrict__ qc,
                                 double* __restrict__ diag, double* __restrict__ b, F32Out fo) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double ih = 1.0 / P.h;
  const double sc = P.dt / (P.h * P.h);
  const double Ssc = 1.0 / P.rho_G - 1.0 / P.rho_L;
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    double an[6];
    bool has[6];
    nbr6(P, a_new, c, i, j, k, an, has);
    const double beta = 1.0 / mix(clamp01(a_new[c]), P.rho_L, P.rho_G);
    const double b32 = (double)(float)beta;
    double d = 0.0, d32 = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        if (has[ax * 2 + sd]) {
          const double bn = 1.0 / mix(clamp01(an[ax * 2 + sd]), P.rho_L, P.rho_G);
          d += sc * 0.5 * (beta + bn);
          d32 += fo.sc * 0.5 * (b32 + (double)(float)bn);
        } else if (pressure_dirichlet(P.kind[ax * 2 + sd])) {
          d += 2.0 * sc * beta;
          d32 += 2.0 * fo.sc * b32;
        }
      }
    const double div = ((us[uidx(P, i + 1, j, k)] - us[uidx(P, i, j, k)]) +
                        (vs[vidx(P, i, j + 1, k)] - vs[vidx(P, i, j, k)]) +
                        (ws[widx(P, i, j, k + 1)] - ws[widx(P, i, j, k)])) * ih;
    qc[c] = beta;
    diag[c] = d;
    b[c] = mdot[c] * Ssc - div;
    if (fo.q) {
      fo.q[c] = (float)beta;
      fo.d[c] = fo.mg ? (float)d32 : (float)d;
    }
  }
}

// ---------------------------------------------------------------- liquid transport velocity
// System D G phi = D u for the divergence-free part u - G phi of the face
// velocities (same boundary kinds as the pressure), written in the pressure
// operator's form with q = 1/dt: (dt/h^2)(1/dt) = 1/h^2 per face.
__global__ void k_div_setup(DevParams P, const double* __restrict__ u, const double* __restrict__ v,
                            const double* __restrict__ w, double* __restrict__ qc, double* __restrict__ diag,
                            double* __restrict__ b, F32Out fo) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double ih = 1.0 / P.h;
  const double ih2 = 1.0 / (P.h * P.h);
  const double q = 1.0 / P.dt, q32 = (double)(float)q;
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    double d = 0.0, d32 = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        if (nbr(P, ax, sd, i, j, k) >= 0) {
          d += ih2;
          d32 += fo.sc * 0.5 * (q32 + q32);
        } else if (pressure_dirichlet(P.kind[ax * 2 + sd])) {
          d += 2.0 * ih2;
          d32 += 2.0 * fo.sc * q32;
        }
      }
    const double div = ((u[uidx(P, i + 1, j, k)] - u[uidx(P, i, j, k)]) + (v[vidx(P, i, j + 1, k)] - v[vidx(P, i, j, k)]) +
                        (w[widx(P, i, j, k + 1)] - w[widx(P, i, j, k)])) * ih;
    if (qc) {   // null: the right-hand side only (the operator is kept from an earlier call)
      qc[c] = q;
      diag[c] = d;
    }
    b[c] = -div;
    if (fo.q) {
      fo.q[c] = (float)q;
      fo.d[c] = fo.mg ? (float)d32 : (float)d;
    }
  }
}

// ---------------------------------------------------------------- S11
// Projected velocity on the face (i, j, k) normal to axis AX, indices in that
// face array (extent +1 along AX).
template <int AX>
__device__ __forceinline__ double project_face(const DevParams& P, const double* __restrict__ a_new,
                                               const double* __restrict__ p, const double* __restrict__ Fs, int i,
                                               int j, int k, double ih) {
  const int fy = P.ny + (AX == 1), fz = P.nz + (AX == 2);
  const long long e = ((long long)i * fy + j) * fz + k;
  const int fpos = AX == 0 ? i : (AX == 1 ? j : k);
  const int nax = AX == 0 ? P.nx : (AX == 1 ? P.ny : P.nz);
  const double us = Fs[e];
  if (fpos == 0 || fpos == nax) {
    const int side = fpos == 0 ? 0 : 1;
    if (!pressure_dirichlet(P.kind[AX * 2 + side])) return us;
    const int ic = AX == 0 ? (side ? i - 1 : i) : i;
    const int jc = AX == 1 ? (side ? j - 1 : j) : j;
    const int kc = AX == 2 ? (side ? k - 1 : k) : k;
    const long long c = cidx(P, ic, jc, kc);
    const double beta = 1.0 / mix(clamp01(a_new[c]), P.rho_L, P.rho_G);
    return side ? us + 2.0 * P.dt * beta * p[c] * ih : us - 2.0 * P.dt * beta * p[c] * ih;
  }
  const int iL = AX == 0 ? i - 1 : i, jL = AX == 1 ? j - 1 : j, kL = AX == 2 ? k - 1 : k;
  const long long cL = cidx(P, iL, jL, kL), cR = cidx(P, i, j, k);
  const double bL = 1.0 / mix(clamp01(a_new[cL]), P.rho_L, P.rho_G);
  const double bR = 1.0 / mix(clamp01(a_new[cR]), P.rho_L, P.rho_G);
  return us - P.dt * 0.5 * (bL + bR) * (p[cR] - p[cL]) * ih;
}

// All three face arrays in one pass over the cells (as the predictor).
__global__ void k_project(DevParams P, const double* __restrict__ a_new, const double* __restrict__ p,
                          const double* __restrict__ us, const double* __restrict__ vs,
                          const double* __restrict__ ws, double* __restrict__ u, double* __restrict__ v,
                          double* __restrict__ w) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double ih = 1.0 / P.h;
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    u[uidx(P, i, j, k)] = project_face<0>(P, a_new, p, us, i, j, k, ih);
    v[vidx(P, i, j, k)] = project_face<1>(P, a_new, p, vs, i, j, k, ih);
    w[widx(P, i, j, k)] = project_face<2>(P, a_new, p, ws, i, j, k, ih);
    if (i == P.nx - 1) u[uidx(P, P.nx, j, k)] = project_face<0>(P, a_new, p, us, P.nx, j, k, ih);
    if (j == P.ny - 1) v[vidx(P, i, P.ny, k)] = project_face<1>(P, a_new, p, vs, i, P.ny, k, ih);
    if (k == P.nz - 1) w[widx(P, i, j, P.nz)] = project_face<2>(P, a_new, p, ws, i, j, P.nz, ih);
  }
}

// ---------------------------------------------------------------- S12
__global__ void k_diagnostics(DevParams P, const double* __restrict__ alpha, const double* __restrict__ c,
                              const double* __restrict__ T, const double* __restrict__ p,
                              const double* __restrict__ mdot, double* partials, unsigned* counter,
                              double* scal) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  double acc[6] = {0.0, 0.0, 0.0, __builtin_inf(), -__builtin_inf(), 0.0};
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    const double a = alpha[e], cv = c[e];
    acc[0] += a;
    acc[1] += P.rho_L * a + cv;
    acc[2] += mdot[e];
    acc[3] = fmin(acc[3], a);
    acc[4] = fmax(acc[4], a);
    const double chk = a + cv + T[e] + p[e];
    if (!isfinite(chk)) acc[5] += 1.0;
  }
  const int ops[6] = {RSUM, RSUM, RSUM, RMIN, RMAX, RSUM};
  if (block_reduce_publish<6>(acc, ops, partials, counter)) {
    double tot[6];
    block_combine<6>(ops, partials, counter, tot);
    if (threadIdx.x == 0) {
      const double v = P.h * P.h * P.h;
      scal[SC_VOL] = v * tot[0];
      scal[SC_FUEL] = v * tot[1];
      scal[SC_MDOT] = v * tot[2];
      scal[SC_AMIN] = tot[3];
      scal[SC_AMAX] = tot[4];
      scal[SC_NONFINITE] = tot[5];
    }
  }
}

// c = rho_G theta omega with theta = max(1 - alpha, theta_min).
__global__ void k_c_from_omega(DevParams P, const double* __restrict__ alpha, const double* __restrict__ omega,
                               double* __restrict__ c) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK)
    c[e] = P.rho_G * fmax(1.0 - clamp01(alpha[e]), P.theta_min) * omega[e];
}

__global__ void k_fill(double* x, double v, long long n) {
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) x[e] = v;
}
__global__ void k_absmax(const double* __restrict__ x, long long n, double* partials, unsigned* counter,
                         double* out) {
  long long b0, b1;
  block_range(n, b0, b1);
  double acc[1] = {0.0};
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    const double v = fabs(x[e]);
    acc[0] = isfinite(v) ? fmax(acc[0], v) : __builtin_inf();
  }
  const int ops[1] = {RMAX};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double tot[1];
    block_combine<1>(ops, partials, counter, tot);
    if (threadIdx.x == 0) *out = tot[0];
  }
}
__global__ void k_scale(double* x, double a, long long n) {
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) x[e] *= a;
}
__global__ void k_int_to_double(const int* s, double* d, long long n) {
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) d[e] = (double)s[e];
}

// ---------------------------------------------------------------- launchers
void launch_xi(const DevParams& P, double* xi, hipStream_t s) {
  k_xi<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, xi);
}
void launch_interface(const DevParams& P, const double* alpha, const double* T, const double* omega,
                      const double* u, const double* v, const double* w, double* mraw, int* adj, int* band,
                      int* band_count, double* partials, unsigned* counter, double* scal, hipStream_t s) {
  const int nb = grid_blocks(P.n);
  const long long cap = ((P.n + nb - 1) / nb + BLOCK - 1) / BLOCK * BLOCK;
  int* off = band_count + MAX_BLOCKS;   // nb + 1 offsets after the counts
  k_interface_scan<false><<<nb, BLOCK, 0, s>>>(P, alpha, mraw, adj, band, band_count);
  k_band_offsets<<<1, 1024, 0, s>>>(band_count, nb, off);
  const int nbi = std::max(NXCD, nb / 8);
  k_interface<<<nbi, BLOCK, 0, s>>>(P, alpha, T, omega, u, v, w, band, off, nb, cap, mraw, adj, partials, counter,
                                    scal);
}
// band_count holds MAX_BLOCKS counts, then MAX_BLOCKS + 1 offsets.
void launch_liquid_saturation(const DevParams& P, const double* alpha, const double* T, double* omega, double* c,
                              int* band, int* band_count, hipStream_t s) {
  const int nb = grid_blocks(P.n);
  const long long cap = ((P.n + nb - 1) / nb + BLOCK - 1) / BLOCK * BLOCK;
  int* off = band_count + MAX_BLOCKS;
  k_interface_scan<true><<<nb, BLOCK, 0, s>>>(P, alpha, nullptr, nullptr, band, band_count);
  k_band_offsets<<<1, 1024, 0, s>>>(band_count, nb, off);
  k_liquid_saturation<<<std::max(NXCD, nb / 8), BLOCK, 0, s>>>(P, alpha, T, band, off, nb, cap, omega, c);
}
long long interface_band_capacity(long long n) {
  const int nb = grid_blocks(n);
  const long long cap = ((n + nb - 1) / nb + BLOCK - 1) / BLOCK * BLOCK;
  return cap * nb;
}
void launch_source(const DevParams& P, const double* alpha, const double* mraw, const double* scal,
                   double* mdot, double* a1, hipStream_t s) {
  k_source<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, alpha, mraw, scal, mdot, a1);
}
void launch_advect(const DevParams& P, const double* a1, const double* omega, const double* T,
                   const double* c, const double* u, const double* v, const double* w, const double* phi,
                   double* a_new, double* c_new, double* T_new, double* partials, unsigned* counter, double* scal,
                   hipStream_t s) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  k_advect<<<nb, BLOCK, 0, s>>>(P, G, a1, omega, T, c, u, v, w, phi, a_new, c_new, T_new, partials, counter, scal);
}
void launch_energy_setup(const DevParams& P, const double* a_new, const double* T_prime,
                         const double* mdot, const double* u, const double* v, const double* w,
                         double* qc, double* diag, double* b, hipStream_t s, F32Out fo) {
  k_energy_setup<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, T_prime, mdot, u, v, w, qc, diag, b, fo);
}
void launch_species_setup(const DevParams& P, const double* a_new, const double* c_prime,
                          const double* mdot, const double* u, const double* v, const double* w,
                          double* qc, double* diag, double* b, double* om0, hipStream_t s, F32Out fo) {
  k_species_setup<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, c_prime, mdot, u, v, w, qc, diag, b, om0, fo);
}
void launch_species_update(const DevParams& P, const double* a_new, const double* c_prime,
                           const double* mdot, const double* om, const double* u, const double* v,
                           const double* w, double* c, double* omega, double* partials,
                           unsigned* counter, double* scal, hipStream_t s) {
  k_species_update<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, c_prime, mdot, om, u, v, w, c, omega, partials, counter, scal);
}
void launch_predictor(const DevParams& P, const double* a_new, const double* xi, const double* u,
                      const double* v, const double* w, double* us, double* vs, double* ws,
                      hipStream_t s) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  k_predictor<<<nb, BLOCK, 0, s>>>(P, G, a_new, xi, u, v, w, us, vs, ws);
}
void launch_pressure_setup(const DevParams& P, const double* a_new, const double* mdot,
                           const double* us, const double* vs, const double* ws, double* qc,
                           double* diag, double* b, hipStream_t s, F32Out fo) {
  k_pressure_setup<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, mdot, us, vs, ws, qc, diag, b, fo);
}
void launch_div_setup(const DevParams& P, const double* u, const double* v, const double* w, double* qc,
                      double* diag, double* b, hipStream_t s, F32Out fo) {
  k_div_setup<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, u, v, w, qc, diag, b, fo);
}
void launch_project(const DevParams& P, const double* a_new, const double* p, const double* us,
                    const double* vs, const double* ws, double* u, double* v, double* w,
                    hipStream_t s) {
  k_project<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, p, us, vs, ws, u, v, w);
}
void launch_diagnostics(const DevParams& P, const double* alpha, const double* c, const double* T,
                        const double* p, const double* mdot, double* partials, unsigned* counter,
                        double* scal, hipStream_t s) {
  k_diagnostics<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, alpha, c, T, p, mdot, partials, counter, scal);
}
void launch_c_from_omega(const DevParams& P, const double* alpha, const double* omega, double* c, hipStream_t s) {
  k_c_from_omega<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, alpha, omega, c);
}
void launch_fill(double* x, double v, long long n, hipStream_t s) {
  k_fill<<<grid_blocks(n), BLOCK, 0, s>>>(x, v, n);
}
void launch_absmax(const double* x, long long n, double* partials, unsigned* counter, double* out, hipStream_t s) {
  k_absmax<<<grid_blocks(n), BLOCK, 0, s>>>(x, n, partials, counter, out);
}
void launch_scale(double* x, double a, long long n, hipStream_t s) {
  k_scale<<<grid_blocks(n), BLOCK, 0, s>>>(x, a, n);
}
void launch_int_to_double(const int* src, double* dst, long long n, hipStream_t s) {
  k_int_to_double<<<grid_blocks(n), BLOCK, 0, s>>>(src, dst, n);
}

}  // namespace dsv
