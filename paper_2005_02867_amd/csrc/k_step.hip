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
// xi = xi0 (Df/2) / max(r, r_fib) at the centre of cell (i, j, k) (eq. 29), centre x0.
__device__ __forceinline__ double xi_at(const DevParams& P, int i, int j, int k) {
  const double x = (i + 0.5) * P.h - P.x0[0], y = (j + 0.5) * P.h - P.x0[1], z = (k + 0.5) * P.h - P.x0[2];
  const double r = sqrt(x * x + y * y + z * z);
  return P.xi0 * (0.5 * P.Df) / fmax(r, P.r_fib);
}
__global__ void __launch_bounds__(BLOCK) k_xi(DevParams P, double* xi) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    xi[c] = xi_at(P, i, j, k);
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
__global__ void __launch_bounds__(BLOCK) k_interface(DevParams P, const double* __restrict__ alpha, const double* __restrict__ T,
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
          jd = rho_gas(P, hit) * P.D * (wsat - wa) / d;
        }
        const double jn = jd + rho_gas(P, hit) * wa * va;
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
__global__ void __launch_bounds__(BLOCK) k_liquid_saturation(DevParams P, const double* __restrict__ alpha, const double* __restrict__ T,
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
__global__ void __launch_bounds__(BLOCK) k_source(DevParams P, const double* __restrict__ alpha, const double* __restrict__ mraw,
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
// H columns at either end of the middle rows.  Positions outside the box
// hold ghost values: alpha1, omega and T repeat the nearest cell of the box
// (so the far-upwind cell of a face next to the box is the upwind cell
// itself: first order there); phi repeats it across walls and changes sign
// across open faces (phi = 0 half a cell outside).
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

// Clamp of a position into [0, n); flips the phi ghost's sign where the
// position left the box across an open face (Dirichlet phi).
__device__ __forceinline__ int clampi(int q, int n) { return q < 0 ? 0 : (q >= n ? n - 1 : q); }
__device__ __forceinline__ double phi_ghost_sign(const DevParams& P, int ax, int q, int n) {
  if (q < 0) return pressure_dirichlet(P.kind[ax * 2]) ? -1.0 : 1.0;
  if (q >= n) return pressure_dirichlet(P.kind[ax * 2 + 1]) ? -1.0 : 1.0;
  return 1.0;
}

// One x-plane of the advection tile in registers: the thread's own centre
// value of each field, then its share of the halo rings.
struct AdvPlane {
  double cA, cO, cT, cP;
  double rA[2], rO[2], rT[2], rP;
};

__device__ __forceinline__ void adv_fetch(const DevParams& P, const double* __restrict__ a1,
                                          const double* __restrict__ omega, const double* __restrict__ T,
                                          const double* __restrict__ phi, int X, bool want, bool want_halo,
                                          int y0, int z0, AdvPlane& f) {
  const long long plane = (long long)P.ny * P.nz;
  const int Xc = clampi(X, P.nx);
  const double sx = phi ? phi_ghost_sign(P, 0, X, P.nx) : 0.0;
  {
    const int ty = threadIdx.x / MZ, tz = threadIdx.x % MZ;
    const int gj = y0 + ty, gk = z0 + tz;   // past the box in a ragged tile: ghosts too
    const long long g = Xc * plane + (long long)clampi(gj, P.ny) * P.nz + clampi(gk, P.nz);
    f.cA = want ? a1[g] : 0.0;
    f.cO = want ? omega[g] : 0.0;
    f.cT = want ? T[g] : 0.0;
    const double sg = phi ? sx * phi_ghost_sign(P, 1, gj, P.ny) * phi_ghost_sign(P, 2, gk, P.nz) : 0.0;
    f.cP = (want && phi) ? sg * phi[g] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int e = threadIdx.x + q * BLOCK;
    int r = 0, c = 0;
    if (e < ARING) ring_entry<2>(e, r, c);
    const bool in = want_halo && e < ARING;
    const long long g = Xc * plane + (long long)clampi(y0 - 2 + r, P.ny) * P.nz + clampi(z0 - 2 + c, P.nz);
    f.rA[q] = in ? a1[g] : 0.0;
    f.rO[q] = in ? omega[g] : 0.0;
    f.rT[q] = in ? T[g] : 0.0;
  }
  {
    const int e = threadIdx.x;
    int r = 0, c = 0;
    if (e < PRING) ring_entry<1>(e, r, c);
    const int gj = y0 - 1 + r, gk = z0 - 1 + c;
    const bool in = phi && want_halo && e < PRING;
    const double sg = in ? sx * phi_ghost_sign(P, 1, gj, P.ny) * phi_ghost_sign(P, 2, gk, P.nz) : 0.0;
    f.rP = in ? sg * phi[Xc * plane + (long long)clampi(gj, P.ny) * P.nz + clampi(gk, P.nz)] : 0.0;
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

// Face velocities and c of the thread's cell in plane X.  Cell indices are
// clamped into the box; the face indices j, k only to the face arrays'
// extent (the row j = ny and the lane k = nz evaluate the high box faces).
struct AdvFaces {
  double u0, u1, v0, v1, w0, w1, c;   // u0: carried from the plane below
  double vx, wx;                      // the tile's extra faces: v above the last row, w above the last lane
};
// Geometric advection: the given liquid fluxes of the faces above (x), below (y, z) and the extra ones.
struct AdvGeoFlux {
  double g1, gv0, gw0, gvx, gwx;
};
__device__ __forceinline__ void adv_faces(const DevParams& P, const double* __restrict__ u,
                                          const double* __restrict__ v, const double* __restrict__ w,
                                          const double* __restrict__ c, int X, bool want, int j, int k,
                                          bool want_vx, bool want_wx, int y0, int z0, AdvFaces& F) {
  const int i = clampi(X, P.nx), jc = clampi(j, P.ny), kc = clampi(k, P.nz);
  const int jf = min(j, P.ny), jf1 = min(j + 1, P.ny), kf = min(k, P.nz), kf1 = min(k + 1, P.nz);
  F.u1 = want ? u[uidx(P, i + 1, jc, kc)] : 0.0;
  F.v0 = want ? v[vidx(P, i, jf, kc)] : 0.0;
  F.v1 = want ? v[vidx(P, i, jf1, kc)] : 0.0;
  F.w0 = want ? w[widx(P, i, jc, kf)] : 0.0;
  F.w1 = want ? w[widx(P, i, jc, kf1)] : 0.0;
  F.c = want ? c[cidx(P, i, jc, kc)] : 0.0;
  // the tile's extra faces: v at row y0 + MY (lane k), w at column z0 + MZ of row y0 + lane (lanes < MY)
  const int lane = threadIdx.x % MZ;
  F.vx = (want && want_vx) ? v[vidx(P, i, min(y0 + MY, P.ny), kc)] : 0.0;
  F.wx = (want && want_wx && lane < MY) ? w[widx(P, i, clampi(y0 + lane, P.ny), min(z0 + MZ, P.nz))] : 0.0;
}
__device__ __forceinline__ void adv_geo_fluxes(const DevParams& P, const double* __restrict__ Fx,
                                               const double* __restrict__ Fy, const double* __restrict__ Fz, int X,
                                               bool want, int j, int k, bool want_vx, bool want_wx, int y0, int z0,
                                               AdvGeoFlux& G) {
  const int i = clampi(X, P.nx), jc = clampi(j, P.ny), kc = clampi(k, P.nz);
  const int jf = min(j, P.ny), kf = min(k, P.nz);
  const int lane = threadIdx.x % MZ;
  G.g1 = want ? Fx[uidx(P, i + 1, jc, kc)] : 0.0;
  G.gv0 = want ? Fy[vidx(P, i, jf, kc)] : 0.0;
  G.gw0 = want ? Fz[widx(P, i, jc, kf)] : 0.0;
  G.gvx = (want && want_vx) ? Fy[vidx(P, i, min(y0 + MY, P.ny), kc)] : 0.0;
  G.gwx = (want && want_wx && lane < MY) ? Fz[widx(P, i, clampi(y0 + lane, P.ny), min(z0 + MZ, P.nz))] : 0.0;
}

// Cell walk of the per-cell setup kernels, marching along x over the same
// tiles (MZ z by MY y rows, one wavefront per row): each thread keeps its
// column's values of the NF fields at x-1, x, x+1 in registers, takes the z
// neighbours from the adjacent lanes (a load only at a wave's first and last
// lane) and loads the y neighbours.  body(c, i, j, k, ctr, nb, has) runs for
// every cell of the box with ctr[f] the cell's value of field f and
// nb[f][0..5] its neighbours at x-1, x+1, y-1, y+1, z-1, z+1 (the cell's own
// value across a box face, where has[] is false).  HIGH = false: the y+1 and
// z+1 entries are not formed (the cell's own value stands there).
template <int NF, bool HIGH = true, class Body>
__device__ __forceinline__ void march_cells(const DevParams& P, const MarchGeom& G,
                                            const double* const (&fld)[NF], Body&& body) {
  const int tz = threadIdx.x % MZ, ty = threadIdx.x / MZ;
  const long long sx = (long long)P.ny * P.nz;
  for (long long t = march_logical(); t < G.tiles; t += gridDim.x) {
    int x0, y0, z0;
    march_tile(G, t, x0, y0, z0);
    const int x1 = min(x0 + G.xlen, P.nx);
    const int j = y0 + ty, k = z0 + tz;
    const bool live = j < P.ny && k < P.nz;
    // rows and lanes past the box hold the nearest cell (their values only feed shuffles no live lane uses)
    const long long col = (long long)min(j, P.ny - 1) * P.nz + min(k, P.nz - 1);
    bool has[6];
    has[2] = j > 0;
    has[3] = j < P.ny - 1;
    has[4] = k > 0;
    has[5] = k < P.nz - 1;
    double xm[NF], xc[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      xc[f] = fld[f][x0 * sx + col];
      xm[f] = x0 > 0 ? fld[f][(x0 - 1) * sx + col] : xc[f];
    }
    for (int x = x0; x < x1; ++x) {
      const long long c = x * sx + col;
      has[0] = x > 0;
      has[1] = x < P.nx - 1;
      double nb[NF][6], xp[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        xp[f] = has[1] ? fld[f][c + sx] : xc[f];
        const double ym = fld[f][has[2] ? c - P.nz : c];
        const double yp = HIGH ? fld[f][has[3] ? c + P.nz : c] : xc[f];
        double zm = __shfl_up(xc[f], 1), zp = HIGH ? __shfl_down(xc[f], 1) : xc[f];
        if (tz == 0) zm = fld[f][has[4] ? c - 1 : c];
        if (HIGH && tz == MZ - 1) zp = fld[f][has[5] ? c + 1 : c];
        nb[f][0] = has[0] ? xm[f] : xc[f];
        nb[f][1] = xp[f];
        nb[f][2] = ym;
        nb[f][3] = yp;
        nb[f][4] = has[4] ? zm : xc[f];
        nb[f][5] = (HIGH && has[5]) ? zp : xc[f];
      }
      if (live) body(c, x, j, k, xc, nb, has);
#pragma unroll
      for (int f = 0; f < NF; ++f) {
        xm[f] = xc[f];
        xc[f] = xp[f];
      }
    }
  }
}

// Van Leer face value on a grid line (cells m, a | b, p; face between a and b)
// for flow in +direction (fwd) or -direction: with C the upwind, D the
// downwind and U the far-upwind cell, C + (C - U)(D - C)/(D - U) where the
// two differences agree in sign, else C.  The reciprocal is the hardware
// estimate refined by two Newton steps (it is only used where D - U is a sum
// of two same-sign differences, never zero).
__device__ __forceinline__ double vl_face(double m, double a, double b, double p, bool fwd) {
  const double C = fwd ? a : b, D = fwd ? b : a, U = fwd ? m : p;
  const double num = (C - U) * (D - C), q = D - U;
  double r = __builtin_amdgcn_rcp(q);
  r = fma(fma(-q, r, 1.0), r, r);
  r = fma(fma(-q, r, 1.0), r, r);
  return num > 0.0 ? fma(num, r, C) : C;
}

// Fluxes (per unit area) through one face: the liquid volume flux F = ul
// alpha_f(ul) with the liquid-transport velocity ul, the vapour mass flux G =
// rho_G omega_f (1 - alpha_f) u and u T_f.  A[], O[], T[] hold the four line
// cells m, a, b, p; box: 0 interior, 1 low box face (b inside), 2 high box
// face (a inside): the face value is the ambient one on inflow (alpha 0,
// omega 0, T_amb), the inside cell's on outflow.  GEO: the liquid flux is
// given (Fl, the geometric advection's) instead.
struct FaceFlux {
  double F, G, uT;
};
template <bool GEO = false>
__device__ __forceinline__ FaceFlux face_flux(const DevParams& P, const double (&A)[4], const double (&O)[4],
                                              const double (&T)[4], double uf, double ul, int box, double Fl = 0.0) {
  const bool fwd = uf > 0.0;
  double af = vl_face(A[0], A[1], A[2], A[3], fwd);
  double of = vl_face(O[0], O[1], O[2], O[3], fwd);
  double al = af;
  const bool fwdl = ul > 0.0;
  if (!GEO && fwdl != fwd) al = vl_face(A[0], A[1], A[2], A[3], fwdl);
  double Tf = 0.0;
  if (P.solve_energy) Tf = vl_face(T[0], T[1], T[2], T[3], fwd);
  if (box) {
    const bool inflow = box == 1 ? fwd : (uf < 0.0);
    const bool inflow_l = box == 1 ? fwdl : (ul < 0.0);
    const double ia = box == 1 ? A[2] : A[1], io = box == 1 ? O[2] : O[1], iT = box == 1 ? T[2] : T[1];
    af = inflow ? 0.0 : ia;
    of = inflow ? 0.0 : io;
    al = inflow_l ? 0.0 : ia;
    Tf = inflow ? P.T_amb : iT;
  }
  return FaceFlux{GEO ? Fl : ul * al, P.rho_G * of * (1.0 - af) * uf, uf * Tf};
}

// Advection of alpha1, c and T (eq. 3 with the liquid-transport velocity,
// the vapour flux and the temperature transport), marching along x.  Each
// face is evaluated once: the x face above a cell is carried to the next
// plane as the one below it; every thread evaluates the y and z faces below
// its cell (dead rows and lanes past the box included, for their
// neighbours), the last row and lane also the faces above; the faces above a
// cell come from the neighbouring row through LDS and from the next lane by a
// shuffle.
template <bool GEO>
__global__ void __launch_bounds__(BLOCK)
k_advect(DevParams P, MarchGeom G, const double* __restrict__ a1, const double* __restrict__ omega,
         const double* __restrict__ T, const double* __restrict__ c, const double* __restrict__ u,
         const double* __restrict__ v, const double* __restrict__ w, const double* __restrict__ phi,
         double* __restrict__ a_new, double* __restrict__ c_new, double* __restrict__ T_new, double* partials,
         unsigned* counter, double* scal, const double* __restrict__ Fx, const double* __restrict__ Fy,
         const double* __restrict__ Fz) {
  __shared__ double sF[3][3][ATILE];      // slot (x mod 3), field (alpha1, omega, T)
  __shared__ double sP[3][PTILE];         // slot, phi
  __shared__ double sY[3][MY + 1][MZ];   // (F, G, uT), y face row, lane
  __shared__ double sZ[3][MY];           // (F, G, uT) of the z face above the last lane, per row
  const int tz = threadIdx.x % MZ, ty = threadIdx.x / MZ;
  const double ih = 1.0 / P.h, s = P.dt / P.h;
  double acc[2] = {0.0, 0.0};   // outward liquid volume flux, vapour mass flux (per area)
  const long long plane = (long long)P.ny * P.nz;
  // The tile's extra faces (the y faces above the last row, the z faces above
  // the last lane of each row) are evaluated by one wave each, chosen by block
  // so that the extra work spreads over the SIMDs.
  const int wave_vx = blockIdx.x % MY, wave_wx = (blockIdx.x + 2) % MY;
  for (long long t = march_logical(); t < G.tiles; t += gridDim.x) {
    int x0, y0, z0;
    march_tile(G, t, x0, y0, z0);
    const int x1 = min(x0 + G.xlen, P.nx);
    const int j = y0 + ty, k = z0 + tz;
    const bool live = j < P.ny && k < P.nz;
    const long long col = live ? (long long)j * P.nz + k : 0;
    // x window of the own column, planes x-1 .. x+2 (ghosts as in the tiles)
    double wA[4], wO[4], wT[4], wP[4];
    __syncthreads();   // the previous tile's last reads of the slots
    AdvPlane f;
    double pA[2], pO[2], pT[2], pP[2];   // planes x0-2, x0-1 (own column only)
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      adv_fetch(P, a1, omega, T, phi, x0 - 2 + q, true, false, y0, z0, f);
      pA[q] = f.cA;
      pO[q] = f.cO;
      pT[q] = f.cT;
      pP[q] = f.cP;
    }
#pragma unroll
    for (int q = 0; q < 3; ++q) {   // planes x0 .. x0+2
      adv_fetch(P, a1, omega, T, phi, x0 + q, x0 + q <= x1 + 1, x0 + q < x1, y0, z0, f);
      adv_store(f, sF[(x0 + q) % 3], sP[(x0 + q) % 3], ty, tz);
      wA[q + 1] = f.cA;
      wO[q + 1] = f.cO;
      wT[q + 1] = f.cT;
      wP[q + 1] = f.cP;
    }
    wA[0] = pA[1];
    wO[0] = pO[1];
    wT[0] = pT[1];
    wP[0] = pP[1];
    AdvFaces F;
    adv_faces(P, u, v, w, c, x0, true, j, k, ty == wave_vx, ty == wave_wx, y0, z0, F);
    AdvGeoFlux FG{};
    if constexpr (GEO) adv_geo_fluxes(P, Fx, Fy, Fz, x0, true, j, k, ty == wave_vx, ty == wave_wx, y0, z0, FG);
    F.u0 = u[uidx(P, x0, clampi(j, P.ny), clampi(k, P.nz))];
    double g0 = GEO ? Fx[uidx(P, x0, clampi(j, P.ny), clampi(k, P.nz))] : 0.0;   // given liquid flux below
    // the x face below plane x0 (cells x0-2 .. x0+1)
    FaceFlux xlo;
    {
      const double ul = phi ? F.u0 - (wP[1] - wP[0]) * ih : F.u0;
      const double A4[4] = {pA[0], pA[1], wA[1], wA[2]}, O4[4] = {pO[0], pO[1], wO[1], wO[2]},
                   T4[4] = {pT[0], pT[1], wT[1], wT[2]};
      xlo = face_flux<GEO>(P, A4, O4, T4, F.u0, ul, x0 == 0 ? 1 : 0, g0);
    }
    __syncthreads();
    int slot = x0 % 3;
    for (int x = x0; x < x1; ++x) {
      AdvPlane nf;
      adv_fetch(P, a1, omega, T, phi, x + 3, x + 3 <= x1 + 1, x + 3 < x1, y0, z0, nf);
      AdvFaces NF;
      adv_faces(P, u, v, w, c, x + 1, x + 1 < x1, j, k, ty == wave_vx, ty == wave_wx, y0, z0, NF);
      AdvGeoFlux NFG{};
      if constexpr (GEO)
        adv_geo_fluxes(P, Fx, Fy, Fz, x + 1, x + 1 < x1, j, k, ty == wave_vx, ty == wave_wx, y0, z0, NFG);
      const double(*S)[ATILE] = sF[slot];
      const double* SP = sP[slot];
      const int ce = (ty + 2) * AHZ + tz + 2, pe = (ty + 1) * PHZ + tz + 1;
      // x face above (cells x-1 .. x+2 of the own column)
      FaceFlux xhi;
      {
        const double ul = phi ? F.u1 - (wP[2] - wP[1]) * ih : F.u1;
        xhi = face_flux<GEO>(P, wA, wO, wT, F.u1, ul, x == P.nx - 1 ? 2 : 0, FG.g1);
      }
      // y faces below the cell (rows j-2 .. j+1 of its column); ce_/pe_ pick
      // the column (tile centre entry) a face is evaluated for
      auto yface = [&](int ce_, int pe_, int r0, double vf, int fpos, double gl) {
        const double A4[4] = {S[0][ce_ + r0 * AHZ], S[0][ce_ + (r0 + 1) * AHZ], S[0][ce_ + (r0 + 2) * AHZ],
                              S[0][ce_ + (r0 + 3) * AHZ]};
        const double O4[4] = {S[1][ce_ + r0 * AHZ], S[1][ce_ + (r0 + 1) * AHZ], S[1][ce_ + (r0 + 2) * AHZ],
                              S[1][ce_ + (r0 + 3) * AHZ]};
        const double T4[4] = {S[2][ce_ + r0 * AHZ], S[2][ce_ + (r0 + 1) * AHZ], S[2][ce_ + (r0 + 2) * AHZ],
                              S[2][ce_ + (r0 + 3) * AHZ]};
        const double ul = phi ? vf - (SP[pe_ + (r0 + 2) * PHZ] - SP[pe_ + (r0 + 1) * PHZ]) * ih : vf;
        return face_flux<GEO>(P, A4, O4, T4, vf, ul, fpos == 0 ? 1 : (fpos == P.ny ? 2 : 0), gl);
      };
      auto zface = [&](int ce_, int pe_, int c0, double wf, int fpos, double gl) {
        const double A4[4] = {S[0][ce_ + c0], S[0][ce_ + c0 + 1], S[0][ce_ + c0 + 2], S[0][ce_ + c0 + 3]};
        const double O4[4] = {S[1][ce_ + c0], S[1][ce_ + c0 + 1], S[1][ce_ + c0 + 2], S[1][ce_ + c0 + 3]};
        const double T4[4] = {S[2][ce_ + c0], S[2][ce_ + c0 + 1], S[2][ce_ + c0 + 2], S[2][ce_ + c0 + 3]};
        const double ul = phi ? wf - (SP[pe_ + c0 + 2] - SP[pe_ + c0 + 1]) * ih : wf;
        return face_flux<GEO>(P, A4, O4, T4, wf, ul, fpos == 0 ? 1 : (fpos == P.nz ? 2 : 0), gl);
      };
      const FaceFlux ylo = yface(ce, pe, -2, F.v0, j, FG.gv0);
      sY[0][ty][tz] = ylo.F;
      sY[1][ty][tz] = ylo.G;
      sY[2][ty][tz] = ylo.uT;
      if (ty == wave_vx) {   // the y faces above the last row (its rows y0+MY-2 .. y0+MY+1)
        const FaceFlux yh = yface((MY + 1) * AHZ + tz + 2, MY * PHZ + tz + 1, -1, F.vx, y0 + MY, FG.gvx);
        sY[0][MY][tz] = yh.F;
        sY[1][MY][tz] = yh.G;
        sY[2][MY][tz] = yh.uT;
      }
      // z faces below the cell (columns k-2 .. k+1); the one above comes from the next lane
      const FaceFlux zlo = zface(ce, pe, -2, F.w0, k, FG.gw0);
      FaceFlux zhi = {__shfl_down(zlo.F, 1, MZ), __shfl_down(zlo.G, 1, MZ), __shfl_down(zlo.uT, 1, MZ)};
      if (ty == wave_wx && tz < MY) {   // lane r: the z face above the last lane of row r
        const FaceFlux zx = zface((tz + 2) * AHZ + MZ + 1, (tz + 1) * PHZ + MZ, -1, F.wx, z0 + MZ, FG.gwx);
        sZ[0][tz] = zx.F;
        sZ[1][tz] = zx.G;
        sZ[2][tz] = zx.uT;
      }
      __syncthreads();   // y and z faces published; every read of this slot is done
      const FaceFlux yhi = {sY[0][ty + 1][tz], sY[1][ty + 1][tz], sY[2][ty + 1][tz]};
      if (tz == MZ - 1) zhi = FaceFlux{sZ[0][ty], sZ[1][ty], sZ[2][ty]};
      __syncthreads();   // every read of the y and z faces is done
      if (live) {
        const double da = (xhi.F - xlo.F) + (yhi.F - ylo.F) + (zhi.F - zlo.F);
        const double dc = (xhi.G - xlo.G) + (yhi.G - ylo.G) + (zhi.G - zlo.G);
        const double T0 = wT[1];
        const long long cc = x * plane + col;
        a_new[cc] = wA[1] - s * da;
        c_new[cc] = F.c - s * dc;
        if (P.solve_energy) {
          const double dT = (xhi.uT - xlo.uT) + (yhi.uT - ylo.uT) + (zhi.uT - zlo.uT) -
                            T0 * ((F.u1 - F.u0) + (F.v1 - F.v0) + (F.w1 - F.w0));
          T_new[cc] = T0 - s * dT;
        } else {
          T_new[cc] = T0;
        }
        // outflow tallies on the box faces of this cell
        if (x == 0) {
          acc[0] -= xlo.F;
          acc[1] -= xlo.G;
        }
        if (x == P.nx - 1) {
          acc[0] += xhi.F;
          acc[1] += xhi.G;
        }
        if (j == 0) {
          acc[0] -= ylo.F;
          acc[1] -= ylo.G;
        }
        if (j == P.ny - 1) {
          acc[0] += yhi.F;
          acc[1] += yhi.G;
        }
        if (k == 0) {
          acc[0] -= zlo.F;
          acc[1] -= zlo.G;
        }
        if (k == P.nz - 1) {
          acc[0] += zhi.F;
          acc[1] += zhi.G;
        }
      }
      adv_store(nf, sF[slot], sP[slot], ty, tz);
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        wA[q] = wA[q + 1];
        wO[q] = wO[q + 1];
        wT[q] = wT[q + 1];
        wP[q] = wP[q + 1];
      }
      wA[3] = nf.cA;
      wO[3] = nf.cO;
      wT[3] = nf.cT;
      wP[3] = nf.cP;
      xlo = xhi;
      NF.u0 = F.u1;
      F = NF;
      if constexpr (GEO) FG = NFG;
      slot = slot == 2 ? 0 : slot + 1;
    }
  }
  advect_publish(P, acc, partials, counter, scal);
}

// ---------------------------------------------------------------- S6-S8
// Energy, eq. 8 after the advection: (rho cp/dt) T - div(k grad T) = (rho cp/dt) T' - mdot dh.
__global__ void __launch_bounds__(BLOCK) k_energy_setup(DevParams P, MarchGeom G, const double* __restrict__ a_new, const double* __restrict__ Tp,
                               const double* __restrict__ mdot, const double* __restrict__ u,
                               const double* __restrict__ v, const double* __restrict__ w,
                               double* __restrict__ qc, double* __restrict__ diag, double* __restrict__ b,
                               F32Out fo) {
  const double ih2 = 1.0 / (P.h * P.h);
  const double Kb = 2.0 * P.k_G * ih2;
  const double* const fl[1] = {a_new};
  march_cells<1>(P, G, fl, [&](long long c, int i, int j, int k, const double (&ctr)[1], const double (&nb)[1][6],
                               const bool (&has)[6]) {
    const double(&an)[6] = nb[0];
    const double ab = clamp01(ctr[0]);
    const double rho = mix(ab, P.rho_L, rho_gas(P, c)), cp = mix(ab, P.cp_L, P.cp_G), kc = mix(ab, P.k_L, P.k_G);
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
  });
}

// Species, eq. 9 for c = rho_G theta omega: (rho_G theta/dt) w - div(rho_G D theta grad w) = c'/dt + mdot
// (without mdot in the literal species form).  Face coefficient K_f = sc (q_c + q_nb)/2 with the cell
// coefficient q = theta and sc = rho_G D/h^2, or, for a variable gas, q = rho_G theta and sc = D/h^2; the
// Dirichlet faces keep the ambient gas's 2 rho_G D/h^2.
// VAR: a variable gas (P.rg set; its density marched beside alpha').
template <bool VAR>
__global__ void __launch_bounds__(BLOCK) k_species_setup(DevParams P, MarchGeom G, const double* __restrict__ a_new, const double* __restrict__ cp_,
                                const double* __restrict__ mdot, const double* __restrict__ u,
                                const double* __restrict__ v, const double* __restrict__ w,
                                double* __restrict__ qc, double* __restrict__ diag, double* __restrict__ b,
                                double* __restrict__ om0, F32Out fo, const double* __restrict__ corr) {
  const double sc = (VAR ? 1.0 : P.rho_G) * P.D / (P.h * P.h);
  const double Kb = 2.0 * P.rho_G * P.D / (P.h * P.h);
  constexpr int NF = VAR ? 2 : 1;   // alpha' (, rho_G)
  const double* fl[NF];
  fl[0] = a_new;
  if constexpr (VAR) fl[NF - 1] = P.rg;
  march_cells<NF>(P, G, fl, [&](long long c, int i, int j, int k, const double (&ctr)[NF], const double (&nb)[NF][6],
                                const bool (&has)[6]) {
    const double(&an)[6] = nb[0];
    const double(&rn)[6] = nb[NF - 1];
    const double th = fmax(1.0 - clamp01(ctr[0]), P.theta_min);
    const double rgc = VAR ? ctr[NF - 1] : P.rho_G;
    const double qcell = VAR ? rgc * th : th;
    double d = rgc * th / P.dt;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        if (has[ax * 2 + sd]) {
          const double tn = fmax(1.0 - clamp01(an[ax * 2 + sd]), P.theta_min);
          d += sc * 0.5 * (qcell + (VAR ? rn[ax * 2 + sd] * tn : tn));
        } else if (scalar_dirichlet(P.kind[ax * 2 + sd], bface_u(P, u, v, w, ax, sd, i, j, k), sd)) {
          d += Kb;
        }
      }
    qc[c] = qcell;
    diag[c] = d;
    // the literal species form has no mdot source (the saturated liquid feeds the gas)
    b[c] = P.species_form == 1 ? cp_[c] / P.dt : cp_[c] / P.dt + mdot[c];
    if (om0) {
      const double w0 = cp_[c] / (rgc * th);
      om0[c] = corr ? w0 + corr[c] : w0;
    }
    if (fo.q) {
      fo.q[c] = (float)qcell;
      fo.d[c] = (float)d;
    }
  });
}

// Flux-form vapour update after the implicit solve; diffusive boundary outflow tally.
template <bool VAR>
__global__ void __launch_bounds__(BLOCK) k_species_update(DevParams P, MarchGeom G, const double* __restrict__ a_new, const double* __restrict__ cp_,
                                 const double* __restrict__ mdot, const double* __restrict__ om,
                                 const double* __restrict__ u, const double* __restrict__ v,
                                 const double* __restrict__ w, double* __restrict__ cout,
                                 double* __restrict__ omega, double* partials, unsigned* counter,
                                 double* scal, double* __restrict__ corr) {
  const double sc = (VAR ? 1.0 : P.rho_G) * P.D / (P.h * P.h);
  const double Kb = 2.0 * P.rho_G * P.D / (P.h * P.h);
  double acc[1] = {0.0};
  constexpr int NF = VAR ? 3 : 2;   // alpha', omega~ (, rho_G)
  const double* fl[NF];
  fl[0] = a_new;
  fl[1] = om;
  if constexpr (VAR) fl[NF - 1] = P.rg;
  march_cells<NF>(P, G, fl, [&](long long c, int i, int j, int k, const double (&ctr)[NF], const double (&nb)[NF][6],
                                const bool (&has)[6]) {
    const double(&an)[6] = nb[0];
    const double(&on)[6] = nb[1];
    const double(&rn)[6] = nb[NF - 1];
    const double th = fmax(1.0 - clamp01(ctr[0]), P.theta_min);
    const double rgc = VAR ? ctr[NF - 1] : P.rho_G;
    const double qcell = VAR ? rgc * th : th;
    const double oc = ctr[1];
    double face = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        if (has[ax * 2 + sd]) {
          const double tn = fmax(1.0 - clamp01(an[ax * 2 + sd]), P.theta_min);
          face += sc * 0.5 * (qcell + (VAR ? rn[ax * 2 + sd] * tn : tn)) * (oc - on[ax * 2 + sd]);
        } else if (scalar_dirichlet(P.kind[ax * 2 + sd], bface_u(P, u, v, w, ax, sd, i, j, k), sd)) {
          face += Kb * oc;
          acc[0] += Kb * oc;
        }
      }
    const double cn = (P.species_form == 1 ? cp_[c] : cp_[c] + P.dt * mdot[c]) - P.dt * face;
    cout[c] = cn;
    omega[c] = cn / (rgc * th);   // a variable gas replaces it from eq. 24 at the end of the step
    if (corr) corr[c] = oc - cp_[c] / (rgc * th);   // the solve's change of the warm start
  });
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
// potential force on the xi jump between the cells L and R either side (gas
// densities gL, gR of those cells).  (i, j, k): the face's indices in its face array.
template <int AX>
__device__ __forceinline__ double predictor_interior(const DevParams& P, double uc, double bn, double fn,
                                                     const double (&vb)[2], const double (&lo)[2],
                                                     const double (&hi)[2], double aL_, double aR_, double gL,
                                                     double gR, double xiL, double xiR, int i, int j, int k,
                                                     double ih) {
  const double back = (uc - bn) * ih, fwd = (fn - uc) * ih;
  double adv = uc * (uc > 0.0 ? back : fwd);
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const double d = (vb[q] > 0.0 ? uc - lo[q] : hi[q] - uc) * ih;
    adv += vb[q] * d;
  }
  const double aL = clamp01(aL_), aR = clamp01(aR_);
  const double rL = mix(aL, P.rho_L, gL), rR = mix(aR, P.rho_L, gR);
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

// Predictor tiles: u, v, w, alpha, xi (and the gas density of a variable
// gas) planes with a halo of 1 (66 x 6, rows y0-1 .. y0+4, columns z0-1 ..
// z0+64); v and w keep their extra face row / column in it.
constexpr int QZ = MZ + 2, QY = MY + 2, QTILE = QZ * QY;

template <int QF>
struct PredPlane {
  double e[QF][2];
};
// Plane X of every field, entries threadIdx.x and threadIdx.x + BLOCK of the
// tile (row-major); X up to xmax (u has nx + 1 planes, the others nx).
template <int QF>
__device__ __forceinline__ void pred_fetch(const DevParams& P, const double* __restrict__ u,
                                           const double* __restrict__ v, const double* __restrict__ w,
                                           const double* __restrict__ a, const double* __restrict__ xi, int X,
                                           int xmax, int y0, int z0, PredPlane<QF>& f) {
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
    if constexpr (QF > 5) f.e[QF - 1][q] = cell ? P.rg[cidx(P, X, gj, gk)] : 0.0;
  }
}
template <int QF>
__device__ __forceinline__ void pred_store(const PredPlane<QF>& f, double (*S)[QTILE]) {
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
// x+1 values; the x-1 values are kept from the previous plane.  Two LDS
// slots: the loads of plane x+2 are issued before plane x is computed and
// land in plane x's slot after it (two barriers per plane), which keeps the
// block at 31.7 KB of LDS (38 KB with the gas density) so that the
// registers, not the LDS, bound the occupancy.  VAR: a variable gas (its density field P.rg rides along as a
// sixth tile).
template <bool VAR>
__global__ void __launch_bounds__(BLOCK)
k_predictor(DevParams P, MarchGeom G, const double* __restrict__ a_new, const double* __restrict__ xi,
            const double* __restrict__ u, const double* __restrict__ v, const double* __restrict__ w,
            double* __restrict__ us, double* __restrict__ vs, double* __restrict__ ws) {
  constexpr int QF = VAR ? 6 : 5;   // u, v, w, alpha, xi (, rho_G)
  __shared__ double sQ[2][QF][QTILE];   // slot ((x - x0) mod 2), field
  const int tz = threadIdx.x % MZ, ty = threadIdx.x / MZ;
  const double ih = 1.0 / P.h;
  constexpr int FU = 0, FV = 1, FW = 2, FA = 3, FX = 4, FR = 5;
  for (long long t = march_logical(); t < G.tiles; t += gridDim.x) {
    int x0, y0, z0;
    march_tile(G, t, x0, y0, z0);
    const int x1 = min(x0 + G.xlen, P.nx);
    const int j = y0 + ty, k = z0 + tz;
    const bool live = j < P.ny && k < P.nz;
    // plane x-1 values of the own column: u, v (j, j+1), w (k, k+1), alpha, xi, rho_G
    double pu, pv0, pv1, pw0, pw1, pa, px, pg;
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
      pg = VAR ? (in ? P.rg[cidx(P, X, jj, kk)] : 0.0) : P.rho_G;
    }
    __syncthreads();   // the previous tile's last reads and writes of the slots
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      PredPlane<QF> f;
      pred_fetch(P, u, v, w, a_new, xi, x0 + q, x1, y0, z0, f);
      pred_store(f, sQ[q]);
    }
    int slot = 0;
    for (int x = x0; x < x1; ++x) {
      PredPlane<QF> nf;
      pred_fetch(P, u, v, w, a_new, xi, x + 2, x1, y0, z0, nf);
      __syncthreads();   // plane x+1 (stored after the previous plane, or before the loop) is visible
      const int s1 = slot ^ 1;
      if (live) {
        const int ce = (ty + 1) * QZ + tz + 1;
        auto T0 = [&](int f, int dy, int dz) { return sQ[slot][f][ce + dy * QZ + dz]; };
        auto T1 = [&](int f, int dy, int dz) { return sQ[s1][f][ce + dy * QZ + dz]; };
        const double uc = T0(FU, 0, 0), vc = T0(FV, 0, 0), wc = T0(FW, 0, 0);
        const double ac = T0(FA, 0, 0), xc = T0(FX, 0, 0);
        auto G0 = [&](int dy, int dz) { return VAR ? T0(FR, dy, dz) : P.rho_G; };
        const double gc = G0(0, 0);
        const double un = T1(FU, 0, 0);   // u(x+1, j, k)
        double ru, rv, rw;
        // u face (x, j, k)
        if (x == 0) {
          ru = predictor_box(P, 0, 0, uc);
        } else {
          const double vb[2] = {0.25 * (pv0 + pv1 + vc + T0(FV, 1, 0)), 0.25 * (pw0 + pw1 + wc + T0(FW, 0, 1))};
          const double lo[2] = {j >= 1 ? T0(FU, -1, 0) : uc, k >= 1 ? T0(FU, 0, -1) : uc};
          const double hi[2] = {j <= P.ny - 2 ? T0(FU, 1, 0) : uc, k <= P.nz - 2 ? T0(FU, 0, 1) : uc};
          ru = predictor_interior<0>(P, uc, pu, un, vb, lo, hi, pa, ac, pg, gc, px, xc, x, j, k, ih);
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
                                     G0(-1, 0), gc, T0(FX, -1, 0), xc, x, j, k, ih);
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
                                     G0(0, -1), gc, T0(FX, 0, -1), xc, x, j, k, ih);
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
        pg = gc;
      }
      __syncthreads();   // every read of this slot is done
      pred_store(nf, sQ[slot]);
      slot = s1;
    }
  }
}

// ---------------------------------------------------------------- S10 setup
// Pressure: sum_f (dt/h^2) (1/rho)_f (p_c - p_nb) = mdot (1/rho_G - 1/rho_L) - div u*.
template <bool VAR>
__global__ void __launch_bounds__(BLOCK) k_pressure_setup(DevParams P, MarchGeom G, const double* __restrict__ a_new, const double* __restrict__ mdot,
                                 const double* __restrict__ us, const double* __restrict__ vs,
                                 const double* __restrict__ ws, double* __restrict__ qc,
                                 double* __restrict__ diag, double* __restrict__ b, F32Out fo,
                                 const double* __restrict__ scomp) {
  const double ih = 1.0 / P.h;
  const double sc = P.dt / (P.h * P.h);
  constexpr int NF = VAR ? 2 : 1;   // alpha' (, rho_G)
  const double* fl[NF];
  fl[0] = a_new;
  if constexpr (VAR) fl[NF - 1] = P.rg;
  march_cells<NF>(P, G, fl, [&](long long c, int i, int j, int k, const double (&ctr)[NF], const double (&nb)[NF][6],
                                const bool (&has)[6]) {
    const double(&an)[6] = nb[0];
    const double(&rn)[6] = nb[NF - 1];
    const double rgc = VAR ? ctr[NF - 1] : P.rho_G;
    const double beta = 1.0 / mix(clamp01(ctr[0]), P.rho_L, rgc);
    const double b32 = (double)(float)beta;
    double d = 0.0, d32 = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        if (has[ax * 2 + sd]) {
          const double bn = 1.0 / mix(clamp01(an[ax * 2 + sd]), P.rho_L, VAR ? rn[ax * 2 + sd] : P.rho_G);
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
    // eq. 7: mdot (1/rho_G - 1/rho_L), less the variable gas's (1 - alpha)(1/rho_G) D rho_G/Dt
    const double src = mdot[c] * (1.0 / rgc - 1.0 / P.rho_L) - (scomp ? scomp[c] : 0.0);
    b[c] = src - div;
    if (fo.q) {
      fo.q[c] = (float)beta;
      fo.d[c] = fo.mg ? (float)d32 : (float)d;
    }
  });
}

// ---------------------------------------------------------------- liquid transport velocity
// System D G phi = D u for the divergence-free part u - G phi of the face
// velocities (same boundary kinds as the pressure), written in the pressure
// operator's form with q = 1/dt: (dt/h^2)(1/dt) = 1/h^2 per face.
// Walks the x-plane tiles: u at the face above a cell is the next plane's
// face below, w above a cell comes from the next lane (lanes past the box
// load the box face's w), only v's two faces are loaded per cell.
__global__ void __launch_bounds__(BLOCK) k_div_setup(DevParams P, MarchGeom G, const double* __restrict__ u, const double* __restrict__ v,
                            const double* __restrict__ w, double* __restrict__ qc, double* __restrict__ diag,
                            double* __restrict__ b, F32Out fo) {
  const double ih = 1.0 / P.h;
  const double ih2 = 1.0 / (P.h * P.h);
  const double q = 1.0 / P.dt, q32 = (double)(float)q;
  const bool op = qc || fo.q;   // the operator is written too
  const int tz = threadIdx.x % MZ, ty = threadIdx.x / MZ;
  const long long sx = (long long)P.ny * P.nz;
  for (long long t = march_logical(); t < G.tiles; t += gridDim.x) {
    int x0, y0, z0;
    march_tile(G, t, x0, y0, z0);
    const int x1 = min(x0 + G.xlen, P.nx);
    const int j = y0 + ty, k = z0 + tz;
    const bool live = j < P.ny && k < P.nz;
    const int jc = min(j, P.ny - 1), kc = min(k, P.nz - 1), kf = min(k, P.nz);
    double u0 = u[uidx(P, x0, jc, kc)];
    for (int x = x0; x < x1; ++x) {
      const double u1 = u[uidx(P, x + 1, jc, kc)];
      const double v0 = v[vidx(P, x, jc, kc)], v1 = v[vidx(P, x, jc + 1, kc)];
      const double w0 = w[widx(P, x, jc, kf)];
      double w1 = __shfl_down(w0, 1);
      if (tz == MZ - 1) w1 = w[widx(P, x, jc, min(k + 1, P.nz))];
      if (live) {
        const long long c = x * sx + (long long)j * P.nz + k;
        if (op) {
          const int pos[3] = {x, j, k}, ext[3] = {P.nx, P.ny, P.nz};
          double d = 0.0, d32 = 0.0;
#pragma unroll
          for (int ax = 0; ax < 3; ++ax)
#pragma unroll
            for (int sd = 0; sd < 2; ++sd) {
              if (sd ? pos[ax] < ext[ax] - 1 : pos[ax] > 0) {
                d += ih2;
                d32 += fo.sc * 0.5 * (q32 + q32);
              } else if (pressure_dirichlet(P.kind[ax * 2 + sd])) {
                d += 2.0 * ih2;
                d32 += 2.0 * fo.sc * q32;
              }
            }
          if (qc) {   // null: the right-hand side only (the operator is kept from an earlier call)
            qc[c] = q;
            diag[c] = d;
          }
          if (fo.q) {
            fo.q[c] = (float)q;
            fo.d[c] = fo.mg ? (float)d32 : (float)d;
          }
        }
        const double div = ((u1 - u0) + (v1 - v0) + (w1 - w0)) * ih;
        b[c] = -div;
      }
      u0 = u1;
    }
  }
}

// ---------------------------------------------------------------- S11
// Projected velocity on the face (i, j, k) normal to axis AX, indices in that
// face array (extent +1 along AX).
template <int AX, bool VAR>
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
    const double beta = 1.0 / mix(clamp01(a_new[c]), P.rho_L, VAR ? P.rg[c] : P.rho_G);
    return side ? us + 2.0 * P.dt * beta * p[c] * ih : us - 2.0 * P.dt * beta * p[c] * ih;
  }
  const int iL = AX == 0 ? i - 1 : i, jL = AX == 1 ? j - 1 : j, kL = AX == 2 ? k - 1 : k;
  const long long cL = cidx(P, iL, jL, kL), cR = cidx(P, i, j, k);
  const double bL = 1.0 / mix(clamp01(a_new[cL]), P.rho_L, VAR ? P.rg[cL] : P.rho_G);
  const double bR = 1.0 / mix(clamp01(a_new[cR]), P.rho_L, VAR ? P.rg[cR] : P.rho_G);
  return us - P.dt * 0.5 * (bL + bR) * (p[cR] - p[cL]) * ih;
}

// All three face arrays in one pass over the cells (as the predictor).
// VAR: a variable gas (its density field P.rg).  DIAG: the step's closing
// diagnostics in the same pass (the sums, extremes and finiteness test of
// k_diagnostics over alpha = a_new, c, T, p and mdot).
template <bool VAR, bool DIAG>
__global__ void __launch_bounds__(BLOCK) k_project(DevParams P, MarchGeom G, const double* __restrict__ a_new, const double* __restrict__ p,
                          const double* __restrict__ us, const double* __restrict__ vs,
                          const double* __restrict__ ws, double* __restrict__ u, double* __restrict__ v,
                          double* __restrict__ w, const double* __restrict__ cf, const double* __restrict__ Tf,
                          const double* __restrict__ mdot, double* partials, unsigned* counter, double* scal) {
  const double ih = 1.0 / P.h;
  double acc[6] = {0.0, 0.0, 0.0, __builtin_inf(), -__builtin_inf(), 0.0};
  // the cell and its neighbour below along each axis (the cell itself at a low box face), walked along x;
  // the faces below the cell as project_face takes them
  constexpr int NF = VAR ? 3 : 2;   // alpha', p (, rho_G)
  const double* fl[NF];
  fl[0] = a_new;
  fl[1] = p;
  if constexpr (VAR) fl[NF - 1] = P.rg;
  march_cells<NF, false>(P, G, fl, [&](long long c, int i, int j, int k, const double (&ctr)[NF],
                                       const double (&nb)[NF][6], const bool (&has)[6]) {
    const long long e[3] = {uidx(P, i, j, k), vidx(P, i, j, k), widx(P, i, j, k)};
    const double fs[3] = {us[e[0]], vs[e[1]], ws[e[2]]};
    const double ac = ctr[0], pc = ctr[1], gc = VAR ? ctr[NF - 1] : P.rho_G;
    double an[3], pn[3], gn[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      an[q] = nb[0][2 * q];
      pn[q] = nb[1][2 * q];
      gn[q] = VAR ? nb[NF - 1][2 * q] : P.rho_G;
    }
    const double bC = 1.0 / mix(clamp01(ac), P.rho_L, gc);
    const int pos[3] = {i, j, k};
    double* const out[3] = {u, v, w};
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      double val;
      if (pos[q] > 0) {
        const double bL = 1.0 / mix(clamp01(an[q]), P.rho_L, gn[q]);
        val = fs[q] - P.dt * 0.5 * (bL + bC) * (pc - pn[q]) * ih;
      } else {
        val = pressure_dirichlet(P.kind[q * 2]) ? fs[q] - 2.0 * P.dt * bC * pc * ih : fs[q];
      }
      out[q][e[q]] = val;
    }
    if (i == P.nx - 1) u[uidx(P, P.nx, j, k)] = project_face<0, VAR>(P, a_new, p, us, P.nx, j, k, ih);
    if (j == P.ny - 1) v[vidx(P, i, P.ny, k)] = project_face<1, VAR>(P, a_new, p, vs, i, P.ny, k, ih);
    if (k == P.nz - 1) w[widx(P, i, j, P.nz)] = project_face<2, VAR>(P, a_new, p, ws, i, j, P.nz, ih);
    if constexpr (DIAG) {
      const double cv = cf[c];
      acc[0] += ac;
      acc[1] += P.rho_L * ac + cv;
      acc[2] += mdot[c];
      acc[3] = fmin(acc[3], ac);
      acc[4] = fmax(acc[4], ac);
      if (!isfinite(ac + cv + Tf[c] + pc)) acc[5] += 1.0;
    }
  });
  if constexpr (DIAG) {
    const int ops[6] = {RSUM, RSUM, RSUM, RMIN, RMAX, RSUM};
    if (block_reduce_publish<6>(acc, ops, partials, counter)) {
      double tot[6];
      block_combine<6>(ops, partials, counter, tot);
      if (threadIdx.x == 0) {
        const double vol = P.h * P.h * P.h;
        scal[SC_VOL] = vol * tot[0];
        scal[SC_FUEL] = vol * tot[1];
        scal[SC_MDOT] = vol * tot[2];
        scal[SC_AMIN] = tot[3];
        scal[SC_AMAX] = tot[4];
        scal[SC_NONFINITE] = tot[5];
      }
    }
  }
}

// ---------------------------------------------------------------- S12
__global__ void __launch_bounds__(BLOCK) k_diagnostics(DevParams P, const double* __restrict__ alpha, const double* __restrict__ c,
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
__global__ void __launch_bounds__(BLOCK) k_c_from_omega(DevParams P, const double* __restrict__ alpha, const double* __restrict__ omega,
                               double* __restrict__ c) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK)
    c[e] = P.rho_G * fmax(1.0 - clamp01(alpha[e]), P.theta_min) * omega[e];
}

__global__ void __launch_bounds__(BLOCK) k_fill(double* x, double v, long long n) {
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) x[e] = v;
}
__global__ void __launch_bounds__(BLOCK) k_absmax(const double* __restrict__ x, long long n, double* partials, unsigned* counter,
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
__global__ void __launch_bounds__(BLOCK) k_scale(double* x, double a, long long n) {
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) x[e] *= a;
}
__global__ void __launch_bounds__(BLOCK) k_int_to_double(const int* s, double* d, long long n) {
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
                   hipStream_t s, const double* Fx, const double* Fy, const double* Fz) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  if (Fx)   // the liquid fluxes are given (geometric advection): no potential tile needed
    k_advect<true><<<nb, BLOCK, 0, s>>>(P, G, a1, omega, T, c, u, v, w, nullptr, a_new, c_new, T_new, partials,
                                        counter, scal, Fx, Fy, Fz);
  else
    k_advect<false><<<nb, BLOCK, 0, s>>>(P, G, a1, omega, T, c, u, v, w, phi, a_new, c_new, T_new, partials,
                                         counter, scal, nullptr, nullptr, nullptr);
}
void launch_energy_setup(const DevParams& P, const double* a_new, const double* T_prime,
                         const double* mdot, const double* u, const double* v, const double* w,
                         double* qc, double* diag, double* b, hipStream_t s, F32Out fo) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  k_energy_setup<<<nb, BLOCK, 0, s>>>(P, G, a_new, T_prime, mdot, u, v, w, qc, diag, b, fo);
}
void launch_species_setup(const DevParams& P, const double* a_new, const double* c_prime,
                          const double* mdot, const double* u, const double* v, const double* w,
                          double* qc, double* diag, double* b, double* om0, hipStream_t s, F32Out fo,
                          const double* corr) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  if (P.rg) k_species_setup<true><<<nb, BLOCK, 0, s>>>(P, G, a_new, c_prime, mdot, u, v, w, qc, diag, b, om0, fo, corr);
  else k_species_setup<false><<<nb, BLOCK, 0, s>>>(P, G, a_new, c_prime, mdot, u, v, w, qc, diag, b, om0, fo, corr);
}
void launch_species_update(const DevParams& P, const double* a_new, const double* c_prime,
                           const double* mdot, const double* om, const double* u, const double* v,
                           const double* w, double* c, double* omega, double* partials,
                           unsigned* counter, double* scal, hipStream_t s, double* corr) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  if (P.rg)
    k_species_update<true><<<nb, BLOCK, 0, s>>>(P, G, a_new, c_prime, mdot, om, u, v, w, c, omega, partials, counter,
                                                scal, corr);
  else
    k_species_update<false><<<nb, BLOCK, 0, s>>>(P, G, a_new, c_prime, mdot, om, u, v, w, c, omega, partials, counter,
                                                 scal, corr);
}
void launch_predictor(const DevParams& P, const double* a_new, const double* xi, const double* u,
                      const double* v, const double* w, double* us, double* vs, double* ws,
                      hipStream_t s) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  if (P.rg) k_predictor<true><<<nb, BLOCK, 0, s>>>(P, G, a_new, xi, u, v, w, us, vs, ws);
  else k_predictor<false><<<nb, BLOCK, 0, s>>>(P, G, a_new, xi, u, v, w, us, vs, ws);
}
void launch_pressure_setup(const DevParams& P, const double* a_new, const double* mdot,
                           const double* us, const double* vs, const double* ws, double* qc,
                           double* diag, double* b, hipStream_t s, F32Out fo, const double* scomp) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  if (P.rg) k_pressure_setup<true><<<nb, BLOCK, 0, s>>>(P, G, a_new, mdot, us, vs, ws, qc, diag, b, fo, scomp);
  else k_pressure_setup<false><<<nb, BLOCK, 0, s>>>(P, G, a_new, mdot, us, vs, ws, qc, diag, b, fo, scomp);
}
void launch_div_setup(const DevParams& P, const double* u, const double* v, const double* w, double* qc,
                      double* diag, double* b, hipStream_t s, F32Out fo) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  k_div_setup<<<nb, BLOCK, 0, s>>>(P, G, u, v, w, qc, diag, b, fo);
}
void launch_project(const DevParams& P, const double* a_new, const double* p, const double* us,
                    const double* vs, const double* ws, double* u, double* v, double* w,
                    hipStream_t s) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  if (P.rg)
    k_project<true, false><<<nb, BLOCK, 0, s>>>(P, G, a_new, p, us, vs, ws, u, v, w, nullptr, nullptr, nullptr,
                                                nullptr, nullptr, nullptr);
  else
    k_project<false, false><<<nb, BLOCK, 0, s>>>(P, G, a_new, p, us, vs, ws, u, v, w, nullptr, nullptr, nullptr,
                                                 nullptr, nullptr, nullptr);
}
void launch_project_diagnostics(const DevParams& P, const double* a_new, const double* p, const double* us,
                                const double* vs, const double* ws, double* u, double* v, double* w,
                                const double* c, const double* T, const double* mdot, double* partials,
                                unsigned* counter, double* scal, hipStream_t s) {
  int nb;
  const MarchGeom G = march_geom(P, nb);
  if (P.rg)
    k_project<true, true><<<nb, BLOCK, 0, s>>>(P, G, a_new, p, us, vs, ws, u, v, w, c, T, mdot, partials, counter,
                                               scal);
  else
    k_project<false, true><<<nb, BLOCK, 0, s>>>(P, G, a_new, p, us, vs, ws, u, v, w, c, T, mdot, partials, counter,
                                                scal);
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
