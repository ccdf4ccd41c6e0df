// Adjoint (reverse-mode) kernels of one step (differentiation form of the
// method of arXiv 2005.02867, Sections 2-3): the transpose of every
// linearised stage of the forward step, in reverse order, for the
// derivative of the liquid volume after a run of steps.
//
// Integer decisions (interface classes and adj, donor/upwind and limiter
// branches, inletOutlet switches, the clamps of the mixing rule) are those of
// the forward step, which is replayed from the stored state before each
// reverse step.  At a kink of a written expression the rule of that
// expression with d|r|/dr = 0 at r = 0 applies (van Leer slope 1 at r = 0).
// Linear solves are differentiated implicitly (the adjoint systems reuse the
// forward operators, all symmetric); the species solve uses the identity
// c^{n+1} = rho_G theta omega~ that holds for an exact solve.
//
// Every kernel gathers (one thread per output cell or face, no floating-point
// atomics), so the reverse sweep is bitwise reproducible.  The interface
// stage, whose band cells feed their adj cell and neighbours, writes each
// band cell's contributions into per-cell records; two gather passes then
// sum them per target in a fixed order.
#include <hip/hip_runtime.h>

#include "ds_device.h"
#include "ds_kernels.h"
#include "ds_stencil.h"
#include "ds_thermo.h"

namespace dsv {

namespace {

__device__ __forceinline__ bool in01(double a) { return a >= 0.0 && a <= 1.0; }
// d theta / d ab for theta = max(1 - ab, theta_min)
__device__ __forceinline__ double dtheta(const DevParams& P, double ab) {
  return (1.0 - ab >= P.theta_min) ? -1.0 : 0.0;
}
// adjoint of alpha' (after advection): its own part plus the property
// clamp's share collected in abar
__device__ __forceinline__ double apbar(const double* A_al, const double* A_ab, const double* a_new, long long c) {
  return A_al[c] + (in01(a_new[c]) ? A_ab[c] : 0.0);
}

// Sum NV per-thread values over the grid and add them to grad[slot[q]].
template <int NV>
__device__ void grad_add(double (&acc)[NV], const int (&slot)[NV], double* partials, unsigned* counter,
                         double* grad) {
  int ops[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) ops[q] = RSUM;
  if (block_reduce_publish<NV>(acc, ops, partials, counter)) {
    double tot[NV];
    block_combine<NV>(ops, partials, counter, tot);
    if (threadIdx.x == 0)
#pragma unroll
      for (int q = 0; q < NV; ++q) grad[slot[q]] += tot[q];
  }
}

// The TVD face value of the forward step (tvd_face, box_face) with its partial derivatives: positions
// along the line of the cells it reads and the derivative for each (a cell
// that appears twice, U := C at the box edge, gets both terms).
struct FaceD {
  double val;
  int pos[3];
  double d[3];
  bool amb;   // inflow boundary face: the ambient value
};

__device__ __forceinline__ FaceD face_deriv(const double* __restrict__ phi, long long line, long long st, int f,
                                            int na, double uf, double amb) {
  FaceD r;
  r.pos[0] = r.pos[1] = r.pos[2] = -1;
  r.d[0] = r.d[1] = r.d[2] = 0.0;
  r.amb = false;
  if (f == 0) {
    if (uf > 0.0) {
      r.val = amb;
      r.amb = true;
    } else {
      r.val = phi[line];
      r.pos[0] = 0;
      r.d[0] = 1.0;
    }
    return r;
  }
  if (f == na) {
    if (uf < 0.0) {
      r.val = amb;
      r.amb = true;
    } else {
      r.val = phi[line + (long long)(na - 1) * st];
      r.pos[0] = na - 1;
      r.d[0] = 1.0;
    }
    return r;
  }
  if (uf == 0.0) {
    r.val = 0.0;
    return r;
  }
  int pc, pd, pu;
  if (uf > 0.0) {
    pc = f - 1;
    pd = f;
    pu = f >= 2 ? f - 2 : pc;
  } else {
    pc = f;
    pd = f - 1;
    pu = f + 1 <= na - 1 ? f + 1 : pc;
  }
  const double C = phi[line + (long long)pc * st], D = phi[line + (long long)pd * st],
               U = phi[line + (long long)pu * st];
  const double den = D - C;
  r.pos[0] = pc;
  if (den == 0.0) {
    r.val = C;
    r.d[0] = 1.0;
    return r;
  }
  const double rr = (C - U) / den;
  const double ar = fabs(rr);
  const double psi = (rr + ar) / (1.0 + ar);
  r.val = C + 0.5 * psi * den;
  const double dpsi = rr > 0.0 ? 2.0 / ((1.0 + rr) * (1.0 + rr)) : (rr == 0.0 ? 1.0 : 0.0);
  r.d[0] = 1.0 - 0.5 * psi + 0.5 * dpsi * (D - U) / den;
  r.pos[1] = pd;
  r.d[1] = 0.5 * psi - 0.5 * dpsi * rr;
  r.pos[2] = pu;
  r.d[2] = -0.5 * dpsi;
  return r;
}

__device__ __forceinline__ double dmatch(const FaceD& f, int p) {
  return (f.pos[0] == p ? f.d[0] : 0.0) + (f.pos[1] == p ? f.d[1] : 0.0) + (f.pos[2] == p ? f.d[2] : 0.0);
}

// Face arrays: index of face (fa along axis ax; cell indices elsewhere).
__device__ __forceinline__ long long fidx(const DevParams& P, int ax, int i, int j, int k) {
  return ax == 0 ? uidx(P, i, j, k) : (ax == 1 ? vidx(P, i, j, k) : widx(P, i, j, k));
}

__device__ __forceinline__ void decode_face(const DevParams& P, int ax, long long e, int& i, int& j, int& k) {
  const int fy = P.ny + (ax == 1), fz = P.nz + (ax == 2);
  decode3(e, fy, fz, i, j, k);
}

// d div_c/d U_e transposed: the adjoint of b = -div(U) at face f of a line
// with cell adjoints lam (interior: (lam_R - lam_L)/h; box faces one-sided).
__device__ __forceinline__ double div_transpose(const DevParams& P, const double* lam, long long line, long long st,
                                                int f, int na) {
  const double lR = f <= na - 1 ? lam[line + (long long)f * st] : 0.0;
  const double lL = f >= 1 ? lam[line + (long long)(f - 1) * st] : 0.0;
  return (lR - lL) / P.h;
}

}  // namespace

// ---------------------------------------------------------------- projection (S11)
// pbar (right-hand side of the adjoint pressure system) and the projection's
// share of abar through beta = 1/rho.
__global__ void __launch_bounds__(BLOCK) k_adj_project(DevParams P, const double* __restrict__ a_new, const double* __restrict__ p,
                              const double* __restrict__ Au, const double* __restrict__ Av,
                              const double* __restrict__ Aw, double* __restrict__ b, double* __restrict__ A_ab,
                              double* partials, unsigned* counter, double* grad) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  double acc[1] = {0.0};
  const double* AU[3] = {Au, Av, Aw};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    const int pos[3] = {i, j, k};
    const int nn[3] = {P.nx, P.ny, P.nz};
    const double ab = clamp01(a_new[c]);
    const double rho = mix(ab, P.rho_L, P.rho_G), beta = 1.0 / rho;
    const double pc = p[c];
    double pbar = 0.0, bbar = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int f = pos[ax] + sd;
        const long long e = fidx(P, ax, ax == 0 ? f : i, ax == 1 ? f : j, ax == 2 ? f : k);
        const double ub = AU[ax][e];
        if (f >= 1 && f <= nn[ax] - 1) {
          const long long nb = nbr(P, ax, sd, i, j, k);
          const double bn = 1.0 / mix(clamp01(a_new[nb]), P.rho_L, P.rho_G);
          const double bf = 0.5 * (beta + bn);
          const double dp = sd ? (p[nb] - pc) : (pc - p[nb]);   // p_R - p_L
          pbar += ub * (sd ? P.dt * bf / P.h : -P.dt * bf / P.h);
          bbar += ub * (-P.dt * 0.5 * dp / P.h);
        } else if (pressure_dirichlet(P.kind[ax * 2 + sd])) {
          pbar += ub * (sd ? 2.0 * P.dt * beta / P.h : -2.0 * P.dt * beta / P.h);
          bbar += ub * (sd ? 2.0 * P.dt * pc / P.h : -2.0 * P.dt * pc / P.h);
        }
      }
    const double ir2 = 1.0 / (rho * rho);
    A_ab[c] = -bbar * (P.rho_L - P.rho_G) * ir2;
    acc[0] += -bbar * (1.0 - ab) * ir2;
    b[c] = pbar;
  }
  const int slot[1] = {GR_RHOG};
  grad_add<1>(acc, slot, partials, counter, grad);
}

// ---------------------------------------------------------------- pressure (S10)
// With lam = A_p^-1 pbar: operator coefficients (beta), source mdot and rho_G.
__global__ void __launch_bounds__(BLOCK) k_adj_pressure(DevParams P, const double* __restrict__ a_new, const double* __restrict__ p,
                               const double* __restrict__ lam, const double* __restrict__ mdot,
                               double* __restrict__ A_ab, double* __restrict__ A_md, double* partials,
                               unsigned* counter, double* grad) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double sc = P.dt / (P.h * P.h);
  const double Ssc = 1.0 / P.rho_G - 1.0 / P.rho_L;
  double acc[1] = {0.0};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    const double ab = clamp01(a_new[c]);
    const double rho = mix(ab, P.rho_L, P.rho_G);
    const double lc = lam[c], pc = p[c];
    double bbar = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const long long nb = nbr(P, ax, sd, i, j, k);
        if (nb >= 0) bbar -= sc * 0.5 * (lc - lam[nb]) * (pc - p[nb]);
        else if (pressure_dirichlet(P.kind[ax * 2 + sd])) bbar -= 2.0 * sc * lc * pc;
      }
    const double ir2 = 1.0 / (rho * rho);
    A_ab[c] += -bbar * (P.rho_L - P.rho_G) * ir2;
    acc[0] += -bbar * (1.0 - ab) * ir2 - lc * mdot[c] / (P.rho_G * P.rho_G);
    A_md[c] = lc * Ssc;
  }
  const int slot[1] = {GR_RHOG};
  grad_add<1>(acc, slot, partials, counter, grad);
}

// ---------------------------------------------------------------- predictor (S9)
namespace {
// 4-point average of component bx on face e (coordinates i, j, k) of
// component AX -- the same expression as the forward predictor.
template <int AX>
__device__ __forceinline__ double pred_vbar(const DevParams& P, int bx, int i, int j, int k, const double* u,
                                            const double* v, const double* w) {
  const int iL = AX == 0 ? i - 1 : i, jL = AX == 1 ? j - 1 : j, kL = AX == 2 ? k - 1 : k;
  if (bx == 0)
    return 0.25 * (u[uidx(P, iL, jL, kL)] + u[uidx(P, iL + 1, jL, kL)] + u[uidx(P, i, j, k)] + u[uidx(P, i + 1, j, k)]);
  if (bx == 1)
    return 0.25 * (v[vidx(P, iL, jL, kL)] + v[vidx(P, iL, jL + 1, kL)] + v[vidx(P, i, j, k)] + v[vidx(P, i, j + 1, k)]);
  return 0.25 * (w[widx(P, iL, jL, kL)] + w[widx(P, iL, jL, kL + 1)] + w[widx(P, i, j, k)] + w[widx(P, i, j, k + 1)]);
}
__device__ __forceinline__ int qslot(int a, int b) { return a * 2 + (b < a ? b : b - 1); }
}  // namespace

// The six transverse-advection weight arrays, passed by value.
struct QPtrs {
  const double* q[6];
};

// Ubar* = Ubar^{n+1} + (transpose of -div) lam_p on every face; the
// transverse-advection weights q_{AX,b} = -dt Ubar* d_b / 4 on interior faces.
template <int AX>
__global__ void __launch_bounds__(BLOCK) k_adj_pred_a(DevParams P, const double* __restrict__ A_U, const double* __restrict__ lam,
                             const double* __restrict__ u, const double* __restrict__ v,
                             const double* __restrict__ w, double* __restrict__ A_Us, double* __restrict__ q0,
                             double* __restrict__ q1) {
  const int fx = P.nx + (AX == 0), fy = P.ny + (AX == 1), fz = P.nz + (AX == 2);
  const long long nf = (long long)fx * fy * fz;
  long long b0, b1;
  block_range(nf, b0, b1);
  const double* F = AX == 0 ? u : (AX == 1 ? v : w);
  const long long sx = (long long)fy * fz, sy = fz, sz = 1;
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    int i, j, k;
    decode3(e, fy, fz, i, j, k);
    const int fpos = AX == 0 ? i : (AX == 1 ? j : k);
    const int nax = AX == 0 ? P.nx : (AX == 1 ? P.ny : P.nz);
    const long long line = AX == 0 ? cidx(P, 0, j, k) : (AX == 1 ? cidx(P, i, 0, k) : cidx(P, i, j, 0));
    const long long cst = AX == 0 ? (long long)P.ny * P.nz : (AX == 1 ? (long long)P.nz : 1);
    const double us = A_U[e] + div_transpose(P, lam, line, cst, fpos, nax);
    A_Us[e] = us;
    double qv[2] = {0.0, 0.0};
    if (fpos >= 1 && fpos <= nax - 1) {
      const double uc = F[e];
      int slot = 0;
#pragma unroll
      for (int bx = 0; bx < 3; ++bx) {
        if (bx == AX) continue;
        const double vb = pred_vbar<AX>(P, bx, i, j, k, u, v, w);
        const int pb = bx == 0 ? i : (bx == 1 ? j : k);
        const int nb_ = bx == 0 ? fx : (bx == 1 ? fy : fz);
        const long long sb = bx == 0 ? sx : (bx == 1 ? sy : sz);
        const double lo = pb >= 1 ? F[e - sb] : uc;
        const double hi = pb <= nb_ - 2 ? F[e + sb] : uc;
        const double d = vb > 0.0 ? (uc - lo) / P.h : (hi - uc) / P.h;
        qv[slot++] = -P.dt * us * d * 0.25;
      }
    }
    q0[e] = qv[0];
    q1[e] = qv[1];
  }
}

// Ubar^n on faces of component AX from the predictor: identity (and the
// copy on open box faces), the transposed same-component advection, and the
// transverse-velocity weights of the other two components.
template <int AX>
__global__ void __launch_bounds__(BLOCK) k_adj_pred_b(DevParams P, const double* __restrict__ A_Us, const double* __restrict__ u,
                             const double* __restrict__ v, const double* __restrict__ w, QPtrs Q,
                             double* __restrict__ A_U) {
  const int fx = P.nx + (AX == 0), fy = P.ny + (AX == 1), fz = P.nz + (AX == 2);
  const long long nf = (long long)fx * fy * fz;
  long long b0, b1;
  block_range(nf, b0, b1);
  const double* F = AX == 0 ? u : (AX == 1 ? v : w);
  const long long sx = (long long)fy * fz, sy = fz, sz = 1;
  const long long sA = AX == 0 ? sx : (AX == 1 ? sy : sz);
  const int nax = AX == 0 ? P.nx : (AX == 1 ? P.ny : P.nz);
  const double ih = 1.0 / P.h;
  for (long long x = b0 + threadIdx.x; x < b1; x += BLOCK) {
    int i, j, k;
    decode3(x, fy, fz, i, j, k);
    const int fpos = AX == 0 ? i : (AX == 1 ? j : k);
    const bool interior = fpos >= 1 && fpos <= nax - 1;
    double acc;
    if (interior) {
      acc = A_Us[x];
    } else {
      const int kind = P.kind[AX * 2 + (fpos == 0 ? 0 : 1)];
      acc = (kind == WALL || kind == INLET) ? 0.0 : A_Us[x];
    }
    double sum = 0.0;   // sum over sources e of Ubar*_e d adv_e / d F_x
    if (interior) {
      // source e = x
      const double uc = F[x];
      double c = uc > 0.0 ? (2.0 * uc - F[x - sA]) / P.h : (F[x + sA] - 2.0 * uc) / P.h;
#pragma unroll
      for (int bx = 0; bx < 3; ++bx) {
        if (bx == AX) continue;
        const double vb = pred_vbar<AX>(P, bx, i, j, k, u, v, w);
        const int pb = bx == 0 ? i : (bx == 1 ? j : k);
        const int nb_ = bx == 0 ? fx : (bx == 1 ? fy : fz);
        if (vb > 0.0) c += pb >= 1 ? vb * ih : 0.0;
        else c += pb <= nb_ - 2 ? -vb * ih : 0.0;
      }
      sum += A_Us[x] * c;
      // sources x +- sb along the transverse axes (same fpos, interior)
#pragma unroll
      for (int bx = 0; bx < 3; ++bx) {
        if (bx == AX) continue;
        const int pb = bx == 0 ? i : (bx == 1 ? j : k);
        const int nb_ = bx == 0 ? fx : (bx == 1 ? fy : fz);
        const long long sb = bx == 0 ? sx : (bx == 1 ? sy : sz);
        if (pb + 1 <= nb_ - 1) {   // e = x + sb: x is its lower neighbour
          const double vb = pred_vbar<AX>(P, bx, bx == 0 ? i + 1 : i, bx == 1 ? j + 1 : j, bx == 2 ? k + 1 : k, u, v, w);
          if (vb > 0.0) sum += A_Us[x + sb] * (-vb * ih);
        }
        if (pb - 1 >= 0) {         // e = x - sb: x is its upper neighbour
          const double vb = pred_vbar<AX>(P, bx, bx == 0 ? i - 1 : i, bx == 1 ? j - 1 : j, bx == 2 ? k - 1 : k, u, v, w);
          if (!(vb > 0.0)) sum += A_Us[x - sb] * (vb * ih);
        }
      }
    }
    // sources x +- sA along the face normal (interior faces only)
    if (fpos + 1 <= nax - 1) {
      const double ue = F[x + sA];
      if (ue > 0.0) sum += A_Us[x + sA] * (-ue * ih);
    }
    if (fpos - 1 >= 1) {
      const double ue = F[x - sA];
      if (!(ue > 0.0)) sum += A_Us[x - sA] * (ue * ih);
    }
    acc += -P.dt * sum;
    // this face inside the 4-point transverse averages of the other components
    const int xc[3] = {i, j, k};
#pragma unroll
    for (int bx = 0; bx < 3; ++bx) {
      if (bx == AX) continue;
      const double* q = Q.q[qslot(bx, AX)];
      const int nAX = nax;
      for (int da = -1; da <= 0; ++da) {
        const int ca = xc[AX] + da;   // cell index along AX of the bx-face
        if (ca < 0 || ca > nAX - 1) continue;
        for (int db = 0; db <= 1; ++db) {
          const int fb = xc[bx] + db;   // face index along bx
          int c3[3] = {xc[0], xc[1], xc[2]};
          c3[AX] = ca;
          c3[bx] = fb;
          acc += q[fidx(P, bx, c3[0], c3[1], c3[2])];
        }
      }
    }
    A_U[x] = acc;
  }
}

// Body forces of the predictor (gravity in p_rgh form, centripetal force):
// their share of abar and rho_G, one thread per cell over its six faces.
__global__ void __launch_bounds__(BLOCK) k_adj_pred_force(DevParams P, const double* __restrict__ a_new, const double* __restrict__ xi,
                                 const double* __restrict__ Usu, const double* __restrict__ Usv,
                                 const double* __restrict__ Usw, double* __restrict__ A_ab, double* partials,
                                 unsigned* counter, double* grad) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double* US[3] = {Usu, Usv, Usw};
  double acc[1] = {0.0};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    const int pos[3] = {i, j, k};
    const int nn[3] = {P.nx, P.ny, P.nz};
    const double ab = clamp01(a_new[c]);
    double abar = 0.0, rbar = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int f = pos[ax] + sd;
        if (f < 1 || f > nn[ax] - 1) continue;
        const int fi = ax == 0 ? f : i, fj = ax == 1 ? f : j, fk = ax == 2 ? f : k;
        const double us = US[ax][fidx(P, ax, fi, fj, fk)];
        const long long nb = nbr(P, ax, sd, i, j, k);
        const long long cL = sd ? c : nb, cR = sd ? nb : c;
        const double aL = clamp01(a_new[cL]), aR = clamp01(a_new[cR]);
        const double rL = mix(aL, P.rho_L, P.rho_G), rR = mix(aR, P.rho_L, P.rho_G);
        const double bf = 0.5 * (1.0 / rL + 1.0 / rR);
        const double xf = (ax == 0 ? fi : fi + 0.5) * P.h - P.x0[0];
        const double yf = (ax == 1 ? fj : fj + 0.5) * P.h - P.x0[1];
        const double zf = (ax == 2 ? fk : fk + 0.5) * P.h - P.x0[2];
        const double gr = P.g[0] * xf + P.g[1] * yf + P.g[2] * zf;
        const double drho = rR - rL;
        const double dF_drho = sd ? (gr / P.h * bf + gr * drho / (2.0 * P.h * rL * rL))
                                  : (-gr / P.h * bf + gr * drho / (2.0 * P.h * rR * rR));
        const double dF_dab = 0.5 * (xi[cR] - xi[cL]) / P.h;
        abar += P.dt * us * (dF_drho * (P.rho_L - P.rho_G) + dF_dab);
        rbar += P.dt * us * dF_drho * (1.0 - ab);
      }
    A_ab[c] += abar;
    acc[0] += rbar;
  }
  const int slot[1] = {GR_RHOG};
  grad_add<1>(acc, slot, partials, counter, grad);
}

// ---------------------------------------------------------------- species (S8)
// Right-hand side of the adjoint species system: omega~bar = omegabar^{n+1}
// + rho_G theta cbar^{n+1} (c^{n+1} = rho_G theta omega~), and the direct
// theta and rho_G shares of c^{n+1}.
__global__ void __launch_bounds__(BLOCK) k_adj_species_rhs(DevParams P, const double* __restrict__ a_new, const double* __restrict__ omt,
                                  const double* __restrict__ A_om, const double* __restrict__ A_c,
                                  double* __restrict__ b, double* __restrict__ A_ab, double* partials,
                                  unsigned* counter, double* grad) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  double acc[1] = {0.0};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    const double ab = clamp01(a_new[c]);
    const double th = fmax(1.0 - ab, P.theta_min);
    const double cb = A_c[c], om = omt[c];
    b[c] = A_om[c] + P.rho_G * th * cb;
    A_ab[c] += P.rho_G * om * cb * dtheta(P, ab);
    acc[0] += th * om * cb;
  }
  const int slot[1] = {GR_RHOG};
  grad_add<1>(acc, slot, partials, counter, grad);
}

// With lam = A_S^-1 omega~bar: cbar' = lam/dt, mdotbar += lam, and the
// operator's derivatives in theta, D and rho_G.
__global__ void __launch_bounds__(BLOCK) k_adj_species(DevParams P, const double* __restrict__ a_new, const double* __restrict__ omt,
                              const double* __restrict__ lam, const double* __restrict__ u,
                              const double* __restrict__ v, const double* __restrict__ w,
                              double* __restrict__ A_ab, double* __restrict__ A_cp, double* __restrict__ A_md,
                              double* partials, unsigned* counter, double* grad) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double ih2 = 1.0 / (P.h * P.h);
  const double sc = P.rho_G * P.D * ih2;
  double acc[2] = {0.0, 0.0};   // D, rho_G
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    const double ab = clamp01(a_new[c]);
    const double th = fmax(1.0 - ab, P.theta_min);
    const double lc = lam[c], xc = omt[c];
    double tbar = -P.rho_G / P.dt * lc * xc;
    double dD = 0.0, Ax = P.rho_G * th / P.dt * xc;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const long long nb = nbr(P, ax, sd, i, j, k);
        if (nb >= 0) {
          const double tn = fmax(1.0 - clamp01(a_new[nb]), P.theta_min);
          const double dl = lc - lam[nb], dx = xc - omt[nb];
          tbar -= sc * 0.5 * dl * dx;
          dD -= 0.5 * P.rho_G * 0.5 * (th + tn) * ih2 * dl * dx;   // each interior face is seen from both cells
          Ax += sc * 0.5 * (th + tn) * dx;
        } else if (scalar_dirichlet(P.kind[ax * 2 + sd], bface_u(P, u, v, w, ax, sd, i, j, k), sd)) {
          dD -= 2.0 * P.rho_G * ih2 * lc * xc;
          Ax += 2.0 * sc * xc;
        }
      }
    A_ab[c] += tbar * dtheta(P, ab);
    A_cp[c] = lc / P.dt;
    A_md[c] += lc;
    acc[0] += dD;
    acc[1] += -lc * Ax / P.rho_G;
  }
  const int slot[2] = {GR_D, GR_RHOG};
  grad_add<2>(acc, slot, partials, counter, grad);
}

// ---------------------------------------------------------------- energy (S7)
// With lam = A_T^-1 Tbar^{n+1}: Tbar' = m lam, mdotbar -= dh lam, the mass
// and conductivity derivatives, dh and T_amb (Dirichlet faces).
__global__ void __launch_bounds__(BLOCK) k_adj_energy(DevParams P, const double* __restrict__ a_new, const double* __restrict__ Tp,
                             const double* __restrict__ Tn, const double* __restrict__ lam,
                             const double* __restrict__ mdot, const double* __restrict__ u,
                             const double* __restrict__ v, const double* __restrict__ w,
                             double* __restrict__ A_ab, double* __restrict__ A_Tp, double* __restrict__ A_md,
                             double* partials, unsigned* counter, double* grad) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double ih2 = 1.0 / (P.h * P.h);
  const double Kb = 2.0 * P.k_G * ih2;
  double acc[3] = {0.0, 0.0, 0.0};   // dh, T_amb, rho_G
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    const double ab = clamp01(a_new[c]);
    const double rho = mix(ab, P.rho_L, P.rho_G), cp = mix(ab, P.cp_L, P.cp_G);
    const double m = rho * cp / P.dt;
    const double lc = lam[c], xc = Tn[c];
    const double mbar = lc * (Tp[c] - xc);
    double kbar = 0.0, tamb = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const long long nb = nbr(P, ax, sd, i, j, k);
        if (nb >= 0) kbar -= ih2 * 0.5 * (lc - lam[nb]) * (xc - Tn[nb]);
        else if (scalar_dirichlet(P.kind[ax * 2 + sd], bface_u(P, u, v, w, ax, sd, i, j, k), sd)) tamb += Kb * lc;
      }
    A_ab[c] += mbar / P.dt * (cp * (P.rho_L - P.rho_G) + rho * (P.cp_L - P.cp_G)) + kbar * (P.k_L - P.k_G);
    A_Tp[c] = m * lc;
    A_md[c] += -P.dh * lc;
    acc[0] += -mdot[c] * lc;
    acc[1] += tamb;
    acc[2] += mbar / P.dt * cp * (1.0 - ab);
  }
  const int slot[3] = {GR_DH, GR_TAMB, GR_RHOG};
  grad_add<3>(acc, slot, partials, counter, grad);
}

// ---------------------------------------------------------------- advection (S5)
// Face part: Ubar from the vapour flux G = rho_G omega_f (1 - alpha_f) u and
// the temperature term u (T_f - T_c); the liquid-velocity adjoint
// Ubar_liq = Fbar alpha_f (or straight into Ubar without the liquid
// transport potential); rho_G and the inflow T_amb.
template <int AX>
__global__ void __launch_bounds__(BLOCK) k_adj_adv_faces(DevParams P, const double* __restrict__ a1, const double* __restrict__ omega,
                                const double* __restrict__ T, const double* __restrict__ uu,
                                const double* __restrict__ phi, const double* __restrict__ a_new,
                                const double* __restrict__ A_al, const double* __restrict__ A_ab,
                                const double* __restrict__ A_cp, const double* __restrict__ A_Tp,
                                double* __restrict__ A_U, double* __restrict__ A_Ul, double* partials,
                                unsigned* counter, double* grad) {
  const int fx = P.nx + (AX == 0), fy = P.ny + (AX == 1), fz = P.nz + (AX == 2);
  const long long nf = (long long)fx * fy * fz;
  long long b0, b1;
  block_range(nf, b0, b1);
  const double sa = P.dt / P.h;
  double acc[2] = {0.0, 0.0};   // rho_G, T_amb
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    int i, j, k;
    decode3(e, fy, fz, i, j, k);
    const int f = AX == 0 ? i : (AX == 1 ? j : k);
    const int na = AX == 0 ? P.nx : (AX == 1 ? P.ny : P.nz);
    const long long line = AX == 0 ? cidx(P, 0, j, k) : (AX == 1 ? cidx(P, i, 0, k) : cidx(P, i, j, 0));
    const long long st = AX == 0 ? (long long)P.ny * P.nz : (AX == 1 ? (long long)P.nz : 1);
    const bool hasL = f >= 1, hasR = f <= na - 1;
    const long long cL = line + (long long)(f - 1) * st, cR = line + (long long)f * st;
    const double uf = uu[e];
    const double apL = hasL ? apbar(A_al, A_ab, a_new, cL) : 0.0, apR = hasR ? apbar(A_al, A_ab, a_new, cR) : 0.0;
    const double cpL = hasL ? A_cp[cL] : 0.0, cpR = hasR ? A_cp[cR] : 0.0;
    const double Fbar = sa * (apR - apL), Gbar = sa * (cpR - cpL);
    const FaceD au = face_deriv(a1, line, st, f, na, uf, 0.0);
    const FaceD om = face_deriv(omega, line, st, f, na, uf, 0.0);
    double ub = Gbar * P.rho_G * om.val * (1.0 - au.val);
    acc[0] += Gbar * om.val * (1.0 - au.val) * uf;
    if (P.solve_energy) {
      const FaceD tf = face_deriv(T, line, st, f, na, uf, P.T_amb);
      const double TpL = hasL ? A_Tp[cL] : 0.0, TpR = hasR ? A_Tp[cR] : 0.0;
      if (hasL) ub += -sa * (tf.val - T[cL]) * TpL;
      if (hasR) ub += sa * (tf.val - T[cR]) * TpR;
      if (tf.amb) acc[1] += sa * uf * (TpR - TpL);
    }
    if (phi) {
      const double ul = liquid_face_u(P, phi, uf, line, st, f, na, AX);
      const FaceD al = face_deriv(a1, line, st, f, na, ul, 0.0);
      A_Ul[e] = Fbar * al.val;
    } else {
      ub += Fbar * au.val;
    }
    A_U[e] += ub;
  }
  const int slot[2] = {GR_RHOG, GR_TAMB};
  grad_add<2>(acc, slot, partials, counter, grad);
}

// Cell part (gather over the faces within two cells along each axis):
// alpha1bar, omegabar^n, Tbar^n (and cbar^n = cbar').
__global__ void __launch_bounds__(BLOCK) k_adj_adv_cells(DevParams P, const double* __restrict__ a1, const double* __restrict__ omega,
                                const double* __restrict__ T, const double* __restrict__ u,
                                const double* __restrict__ v, const double* __restrict__ w,
                                const double* __restrict__ phi, const double* __restrict__ a_new,
                                const double* __restrict__ A_al, const double* __restrict__ A_ab,
                                const double* __restrict__ A_cp, const double* __restrict__ A_Tp,
                                double* __restrict__ A_a1, double* __restrict__ A_om, double* __restrict__ A_T,
                                double* __restrict__ A_c) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double sa = P.dt / P.h;
  for (long long cc = b0 + threadIdx.x; cc < b1; cc += BLOCK) {
    int i, j, k;
    decode(P, cc, i, j, k);
    const int pos[3] = {i, j, k};
    const int nn[3] = {P.nx, P.ny, P.nz};
    const long long st[3] = {(long long)P.ny * P.nz, (long long)P.nz, 1};
    const long long line[3] = {cc - (long long)i * st[0], cc - (long long)j * st[1], cc - (long long)k};
    // alpha' = alpha1 - (dt/h) sum of flux differences: identity plus the flux terms
    double a1b = apbar(A_al, A_ab, a_new, cc), omb = 0.0, Tb = 0.0;
    if (P.solve_energy) {
      const double du = (u[uidx(P, i + 1, j, k)] - u[uidx(P, i, j, k)]) + (v[vidx(P, i, j + 1, k)] - v[vidx(P, i, j, k)]) +
                        (w[widx(P, i, j, k + 1)] - w[widx(P, i, j, k)]);
      Tb = A_Tp[cc] * (1.0 + sa * du);
    }
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int na = nn[ax], me = pos[ax];
      for (int f = me - 1; f <= me + 2; ++f) {
        if (f < 0 || f > na) continue;
        const double uf = ax == 0 ? u[uidx(P, f, j, k)] : (ax == 1 ? v[vidx(P, i, f, k)] : w[widx(P, i, j, f)]);
        const bool hasL = f >= 1, hasR = f <= na - 1;
        const long long cL = line[ax] + (long long)(f - 1) * st[ax], cR = line[ax] + (long long)f * st[ax];
        const double apL = hasL ? apbar(A_al, A_ab, a_new, cL) : 0.0, apR = hasR ? apbar(A_al, A_ab, a_new, cR) : 0.0;
        const double cpL = hasL ? A_cp[cL] : 0.0, cpR = hasR ? A_cp[cR] : 0.0;
        const double Fbar = sa * (apR - apL), Gbar = sa * (cpR - cpL);
        const FaceD au = face_deriv(a1, line[ax], st[ax], f, na, uf, 0.0);
        const FaceD om = face_deriv(omega, line[ax], st[ax], f, na, uf, 0.0);
        omb += Gbar * P.rho_G * (1.0 - au.val) * uf * dmatch(om, me);
        a1b += -Gbar * P.rho_G * om.val * uf * dmatch(au, me);
        if (phi) {
          const double ul = liquid_face_u(P, phi, uf, line[ax], st[ax], f, na, ax);
          const FaceD al = face_deriv(a1, line[ax], st[ax], f, na, ul, 0.0);
          a1b += Fbar * ul * dmatch(al, me);
        } else {
          a1b += Fbar * uf * dmatch(au, me);
        }
        if (P.solve_energy) {
          const double TpL = hasL ? A_Tp[cL] : 0.0, TpR = hasR ? A_Tp[cR] : 0.0;
          const FaceD tf = face_deriv(T, line[ax], st[ax], f, na, uf, P.T_amb);
          Tb += sa * uf * (TpR - TpL) * dmatch(tf, me);
        }
      }
    }
    A_a1[cc] = a1b;
    A_om[cc] = omb;
    if (P.solve_energy) A_T[cc] = Tb;
    A_c[cc] = A_cp[cc];
  }
}

// Right-hand side of the adjoint liquid-transport potential system:
// phibar from Ubar_liq (u_liq = u - G phi, phi = 0 half a cell outside open faces).
__global__ void __launch_bounds__(BLOCK) k_adj_phi_rhs(DevParams P, const double* __restrict__ Ulu, const double* __restrict__ Ulv,
                              const double* __restrict__ Ulw, double* __restrict__ b) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double* UL[3] = {Ulu, Ulv, Ulw};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    int i, j, k;
    decode(P, c, i, j, k);
    const int pos[3] = {i, j, k};
    const int nn[3] = {P.nx, P.ny, P.nz};
    double s = 0.0;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax)
#pragma unroll
      for (int sd = 0; sd < 2; ++sd) {
        const int f = pos[ax] + sd;
        const double ul = UL[ax][fidx(P, ax, ax == 0 ? f : i, ax == 1 ? f : j, ax == 2 ? f : k)];
        if (f >= 1 && f <= nn[ax] - 1) s += sd ? ul / P.h : -ul / P.h;
        else if (pressure_dirichlet(P.kind[ax * 2 + sd])) s += sd ? 2.0 * ul / P.h : -2.0 * ul / P.h;
      }
    b[c] = s;
  }
}

// Ubar += Ubar_liq + (transpose of -div) lam_phi.
template <int AX>
__global__ void __launch_bounds__(BLOCK) k_adj_phi_faces(DevParams P, const double* __restrict__ A_Ul, const double* __restrict__ lam,
                                double* __restrict__ A_U) {
  const int fx = P.nx + (AX == 0), fy = P.ny + (AX == 1), fz = P.nz + (AX == 2);
  const long long nf = (long long)fx * fy * fz;
  long long b0, b1;
  block_range(nf, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    int i, j, k;
    decode3(e, fy, fz, i, j, k);
    const int f = AX == 0 ? i : (AX == 1 ? j : k);
    const int na = AX == 0 ? P.nx : (AX == 1 ? P.ny : P.nz);
    const long long line = AX == 0 ? cidx(P, 0, j, k) : (AX == 1 ? cidx(P, i, 0, k) : cidx(P, i, j, 0));
    const long long st = AX == 0 ? (long long)P.ny * P.nz : (AX == 1 ? (long long)P.nz : 1);
    A_U[e] += A_Ul[e] + div_transpose(P, lam, line, st, f, na);
  }
}

// ---------------------------------------------------------------- source (eq. 4) and redistribution (eqs. 19-21)
// alphabar^n = alpha1bar, mdotbar -= dt alpha1bar / rho_L, and
// Kbar = sum mdotbar f mraw -> S1bar = Kbar/S2, S2bar = -Kbar S1/S2^2.
__global__ void __launch_bounds__(BLOCK) k_adj_source(DevParams P, const double* __restrict__ alpha, const double* __restrict__ mraw,
                             const double* __restrict__ A_a1, double* __restrict__ A_md,
                             double* __restrict__ A_al, const double* __restrict__ scal, double* partials,
                             unsigned* counter, double* grad) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  double acc[1] = {0.0};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    const double a1b = A_a1[c];
    const double md = A_md[c] - P.dt / P.rho_L * a1b;
    A_md[c] = md;
    A_al[c] = a1b;
    const double a = alpha[c];
    const double f = sqrt(fmax(a * (1.0 - a), 0.0));
    acc[0] += md * f * mraw[c];
  }
  int ops[1] = {RSUM};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double tot[1];
    block_combine<1>(ops, partials, counter, tot);
    if (threadIdx.x == 0) {
      const double S1 = scal[SC_S1], S2 = scal[SC_S2];
      grad[GR_S1B] = S2 != 0.0 ? tot[0] / S2 : 0.0;
      grad[GR_S2B] = S2 != 0.0 ? -tot[0] * S1 / (S2 * S2) : 0.0;
    }
  }
}

// ---------------------------------------------------------------- interface flux (S1-S3)
// Band cells with an adj: mdotbar -> mrawbar (through K and f), then the
// flux j.n at adj (eqs. 12-14, 17): omega_sat(T_int) (T, dh), omega_adj,
// the adj cell velocity, the normal and |grad alpha| (six alpha neighbours),
// D and rho_G.  The band cell's own alpha and T terms are added in place;
// what goes to other cells is recorded: R.gb[q] (to alpha of the neighbours
// +-q), R.om (to omega of adj), R.f[q] (to each of adj's two q faces), and
// adj is marked in R.hit (the first band cell to mark it also lists it), its
// march distance maxed into R.rmax.
__global__ void __launch_bounds__(BLOCK) k_adj_interface(DevParams P, const double* __restrict__ alpha, const double* __restrict__ T,
                                const double* __restrict__ omega, const double* __restrict__ u,
                                const double* __restrict__ v, const double* __restrict__ w,
                                const double* __restrict__ mraw, const int* __restrict__ adj,
                                const double* __restrict__ A_md, const double* __restrict__ scal,
                                double* __restrict__ A_al, double* __restrict__ A_T, IfaceRecords R,
                                double* partials, unsigned* counter, double* grad) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double K = scal[SC_K];
  const double S1b = grad[GR_S1B], S2b = grad[GR_S2B];
  double acc[3] = {0.0, 0.0, 0.0};   // D, dh, rho_G
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    const int hit = adj[c];
    if (hit < 0) continue;
    int i, j, k;
    decode(P, c, i, j, k);
    const double a = alpha[c];
    const double f = sqrt(fmax(a * (1.0 - a), 0.0));
    const double m = mraw[c];
    const double md = A_md[c];
    const double mb = md * K * f + S1b + S2b * f;
    const double fb = md * K * m + S2b * m;
    if (f > 0.0) A_al[c] += fb * (1.0 - 2.0 * a) / (2.0 * f);
    // geometry (same values as the forward)
    const double dx = __dsub_rn(alpha_or0(P, alpha, i + 1, j, k), alpha_or0(P, alpha, i - 1, j, k));
    const double dy = __dsub_rn(alpha_or0(P, alpha, i, j + 1, k), alpha_or0(P, alpha, i, j - 1, k));
    const double dz = __dsub_rn(alpha_or0(P, alpha, i, j, k + 1), alpha_or0(P, alpha, i, j, k - 1));
    const double nrm = __dsqrt_rn(__dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz)));
    const double n[3] = {__ddiv_rn(-dx, nrm), __ddiv_rn(-dy, nrm), __ddiv_rn(-dz, nrm)};
    int ti, tj, tk;
    decode(P, hit, ti, tj, tk);
    const double di = ti - i, dj = tj - j, dk = tk - k;
    const double d = P.h * sqrt(di * di + dj * dj + dk * dk);
    double dydT, dydh;
    const double y = equilibrium_y_grad(P, T[c], dydT, dydh);
    const double ws = mass_fraction(P, y);
    const double den = y * P.M_v + (1.0 - y) * P.M_G;
    const double dws_dy = P.M_v * P.M_G / (den * den);
    const double wa = omega[hit];
    const long long fu[2] = {uidx(P, ti, tj, tk), uidx(P, ti + 1, tj, tk)};
    const long long fv[2] = {vidx(P, ti, tj, tk), vidx(P, ti, tj + 1, tk)};
    const long long fw[2] = {widx(P, ti, tj, tk), widx(P, ti, tj, tk + 1)};
    const double vc[3] = {0.5 * (u[fu[0]] + u[fu[1]]), 0.5 * (v[fv[0]] + v[fv[1]]), 0.5 * (w[fw[0]] + w[fw[1]])};
    const double va = vc[0] * n[0] + vc[1] * n[1] + vc[2] * n[2];
    const double jn = P.rho_G * P.D * (ws - wa) / d + P.rho_G * wa * va;
    const double gm = nrm / (2.0 * P.h);
    const double jb = mb * gm;
    const double nrmb = mb * jn / (2.0 * P.h);
    const double wsb = jb * P.rho_G * P.D / d;
    A_T[c] += wsb * dws_dy * dydT;
    acc[1] += wsb * dws_dy * dydh;
    acc[0] += jb * P.rho_G * (ws - wa) / d;
    acc[2] += jb * jn / P.rho_G;
    R.om[c] = jb * P.rho_G * (va - P.D / d);
    const double vab = jb * P.rho_G * wa;
    R.f[0][c] = 0.5 * vab * n[0];
    R.f[1][c] = 0.5 * vab * n[1];
    R.f[2][c] = 0.5 * vab * n[2];
    // 0x3FF0000000000000 is 1.0: the cell is listed by whichever band cell marks it first
    if (atomicCAS(reinterpret_cast<unsigned long long*>(R.hit) + hit, 0ull, 0x3FF0000000000000ull) == 0ull)
      R.list[atomicAdd(R.nlist, 1u)] = hit;
    const int dist = max(abs(ti - i), max(abs(tj - j), abs(tk - k)));
    atomicMax(R.rmax, (unsigned)dist);
    const double nb[3] = {vab * vc[0], vab * vc[1], vab * vc[2]};
    const double ndot = nb[0] * n[0] + nb[1] * n[1] + nb[2] * n[2];
    double gb[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) gb[q] = -(nb[q] - n[q] * ndot) / nrm - nrmb * n[q];
#pragma unroll
    for (int q = 0; q < 3; ++q) R.gb[q][c] = gb[q];
  }
  const int slot[3] = {GR_D, GR_DH, GR_RHOG};
  grad_add<3>(acc, slot, partials, counter, grad);
}

// Before the interface stage: no cell is an adj yet, march distance 0, the
// list empty.
__global__ void __launch_bounds__(BLOCK) k_adj_iface_clear(DevParams P, IfaceRecords R) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) R.hit[e] = 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *R.rmax = 0u;
    *R.nlist = 0u;
  }
}

// Gather of the interface records to alpha, per cell e in a fixed order:
// from the band neighbours' gb (the lower neighbour along q adds gb[q], the
// upper one subtracts it).
__global__ void __launch_bounds__(BLOCK) k_adj_iface_gather(DevParams P, const int* __restrict__ adj, IfaceRecords R,
                                   double* __restrict__ A_al) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  const long long st[3] = {(long long)P.ny * P.nz, (long long)P.nz, 1};
  const int nn[3] = {P.nx, P.ny, P.nz};
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    int i, j, k;
    decode(P, e, i, j, k);
    const int pos[3] = {i, j, k};
    double acc = 0.0;
    bool any = false;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      if (pos[q] > 0 && adj[e - st[q]] >= 0) {
        acc += R.gb[q][e - st[q]];
        any = true;
      }
      if (pos[q] < nn[q] - 1 && adj[e + st[q]] >= 0) {
        acc -= R.gb[q][e + st[q]];
        any = true;
      }
    }
    if (any) A_al[e] += acc;
  }
}

// Gather to the adj cells, one wavefront per listed cell e: omega of e from
// every band cell within the largest march distance whose adj is e, and the
// sums of their face records, kept for the face pass.  Lane l takes the
// cells l, l + 64, ... of the cube around e in i, j, k order, and the lanes'
// sums meet in a fixed shuffle tree: the result does not depend on the
// order of the list.
__global__ void __launch_bounds__(BLOCK) k_adj_iface_targets(DevParams P, const int* __restrict__ adj, IfaceRecords R,
                                    double* __restrict__ A_om) {
  const int rm = (int)*R.rmax;
  const unsigned nl = *R.nlist;
  const int lane = threadIdx.x & 63;
  const unsigned nwave = gridDim.x * (BLOCK / 64);
  const int side = 2 * rm + 1;
  const int cube = side * side * side;
  for (unsigned t = blockIdx.x * (BLOCK / 64) + threadIdx.x / 64; t < nl; t += nwave) {
    const int e = R.list[t];
    int i, j, k;
    decode(P, e, i, j, k);
    double som = 0.0, sf[3] = {0.0, 0.0, 0.0};
    for (int q = lane; q < cube; q += 64) {
      const int ci = i + q / (side * side) - rm, cj = j + (q / side) % side - rm, ck = k + q % side - rm;
      if (ci < 0 || ci >= P.nx || cj < 0 || cj >= P.ny || ck < 0 || ck >= P.nz) continue;
      const long long c = cidx(P, ci, cj, ck);
      if (adj[c] != e) continue;
      som += R.om[c];
#pragma unroll
      for (int a = 0; a < 3; ++a) sf[a] += R.f[a][c];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      som += __shfl_down(som, off, 64);
#pragma unroll
      for (int a = 0; a < 3; ++a) sf[a] += __shfl_down(sf[a], off, 64);
    }
    if (lane == 0) {
      A_om[e] += som;
#pragma unroll
      for (int a = 0; a < 3; ++a) R.gsf[a][e] = sf[a];
    }
  }
}

// Face pass: each face of an adj cell gets that cell's face sum; a face
// between two adj cells gets the lower one's, then the upper one's.  The
// thread of the cell below a face (of the cell above, for a low box face)
// writes it.
__global__ void __launch_bounds__(BLOCK) k_adj_iface_faces(DevParams P, IfaceRecords R, double* __restrict__ Au, double* __restrict__ Av,
                                  double* __restrict__ Aw) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  double* const AU[3] = {Au, Av, Aw};
  const long long st[3] = {(long long)P.ny * P.nz, (long long)P.nz, 1};
  const int nn[3] = {P.nx, P.ny, P.nz};
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    int i, j, k;
    decode(P, e, i, j, k);
    const int pos[3] = {i, j, k};
    const bool me = R.hit[e] != 0.0;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const long long lo = q == 0 ? uidx(P, i, j, k) : (q == 1 ? vidx(P, i, j, k) : widx(P, i, j, k));
      const long long hi = q == 0 ? uidx(P, i + 1, j, k) : (q == 1 ? vidx(P, i, j + 1, k) : widx(P, i, j, k + 1));
      if (pos[q] == 0 && me) AU[q][lo] += R.gsf[q][e];
      const bool up = pos[q] < nn[q] - 1 && R.hit[e + st[q]] != 0.0;
      if (me && up) AU[q][hi] += R.gsf[q][e] + R.gsf[q][e + st[q]];
      else if (me) AU[q][hi] += R.gsf[q][e];
      else if (up) AU[q][hi] += R.gsf[q][e + st[q]];
    }
  }
}

// ---------------------------------------------------------------- initial vapour c^0 = rho_G theta omega^0
__global__ void __launch_bounds__(BLOCK) k_adj_init_c(DevParams P, const double* __restrict__ alpha, const double* __restrict__ omega,
                             const double* __restrict__ A_c, double* __restrict__ A_al, double* __restrict__ A_om,
                             double* partials, unsigned* counter, double* grad) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  double acc[1] = {0.0};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    const double a = alpha[c];
    const double ab = clamp01(a);
    const double th = fmax(1.0 - ab, P.theta_min);
    const double cb = A_c[c];
    A_om[c] += P.rho_G * th * cb;
    if (in01(a)) A_al[c] += P.rho_G * omega[c] * cb * dtheta(P, ab);
    acc[0] += th * omega[c] * cb;
  }
  const int slot[1] = {GR_RHOG};
  grad_add<1>(acc, slot, partials, counter, grad);
}

// ---------------------------------------------------------------- launchers
void launch_adj_project(const DevParams& P, const double* a_new, const double* p, double* const AU[3], double* b,
                        double* A_ab, double* partials, unsigned* counter, double* grad, hipStream_t s) {
  k_adj_project<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, p, AU[0], AU[1], AU[2], b, A_ab, partials, counter, grad);
}
void launch_adj_pressure(const DevParams& P, const double* a_new, const double* p, const double* lam,
                         const double* mdot, double* A_ab, double* A_md, double* partials, unsigned* counter,
                         double* grad, hipStream_t s) {
  k_adj_pressure<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, p, lam, mdot, A_ab, A_md, partials, counter, grad);
}
void launch_adj_predictor(const DevParams& P, const double* a_new, const double* xi, double* const AU[3],
                          double* const AUs[3], double* const Q[6], const double* lam,
                          const double* u, const double* v, const double* w, double* A_ab, double* partials,
                          unsigned* counter, double* grad, hipStream_t s) {
  const long long nu = (long long)(P.nx + 1) * P.ny * P.nz, nv = (long long)P.nx * (P.ny + 1) * P.nz,
                  nw = (long long)P.nx * P.ny * (P.nz + 1);
  k_adj_pred_a<0><<<grid_blocks(nu), BLOCK, 0, s>>>(P, AU[0], lam, u, v, w, AUs[0], Q[0], Q[1]);
  k_adj_pred_a<1><<<grid_blocks(nv), BLOCK, 0, s>>>(P, AU[1], lam, u, v, w, AUs[1], Q[2], Q[3]);
  k_adj_pred_a<2><<<grid_blocks(nw), BLOCK, 0, s>>>(P, AU[2], lam, u, v, w, AUs[2], Q[4], Q[5]);
  QPtrs qp;
  for (int q = 0; q < 6; ++q) qp.q[q] = Q[q];
  k_adj_pred_b<0><<<grid_blocks(nu), BLOCK, 0, s>>>(P, AUs[0], u, v, w, qp, AU[0]);
  k_adj_pred_b<1><<<grid_blocks(nv), BLOCK, 0, s>>>(P, AUs[1], u, v, w, qp, AU[1]);
  k_adj_pred_b<2><<<grid_blocks(nw), BLOCK, 0, s>>>(P, AUs[2], u, v, w, qp, AU[2]);
  k_adj_pred_force<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, xi, AUs[0], AUs[1], AUs[2], A_ab, partials, counter,
                                                      grad);
}
void launch_adj_species_rhs(const DevParams& P, const double* a_new, const double* omt, const double* A_om,
                            const double* A_c, double* b, double* A_ab, double* partials, unsigned* counter,
                            double* grad, hipStream_t s) {
  k_adj_species_rhs<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, omt, A_om, A_c, b, A_ab, partials, counter, grad);
}
void launch_adj_species(const DevParams& P, const double* a_new, const double* omt, const double* lam,
                        const double* u, const double* v, const double* w, double* A_ab, double* A_cp, double* A_md,
                        double* partials, unsigned* counter, double* grad, hipStream_t s) {
  k_adj_species<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, omt, lam, u, v, w, A_ab, A_cp, A_md, partials, counter,
                                                   grad);
}
void launch_adj_energy(const DevParams& P, const double* a_new, const double* Tp, const double* Tn, const double* lam,
                       const double* mdot, const double* u, const double* v, const double* w, double* A_ab,
                       double* A_Tp, double* A_md, double* partials, unsigned* counter, double* grad,
                       hipStream_t s) {
  k_adj_energy<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a_new, Tp, Tn, lam, mdot, u, v, w, A_ab, A_Tp, A_md, partials,
                                                  counter, grad);
}
void launch_adj_advect(const DevParams& P, const double* a1, const double* omega, const double* T, const double* u,
                       const double* v, const double* w, const double* phi, const double* a_new, const double* A_al,
                       const double* A_ab, const double* A_cp, const double* A_Tp, double* const AU[3],
                       double* const AUl[3], double* A_a1, double* A_om, double* A_T, double* A_c, double* partials,
                       unsigned* counter, double* grad, hipStream_t s) {
  const long long nu = (long long)(P.nx + 1) * P.ny * P.nz, nv = (long long)P.nx * (P.ny + 1) * P.nz,
                  nw = (long long)P.nx * P.ny * (P.nz + 1);
  k_adj_adv_faces<0><<<grid_blocks(nu), BLOCK, 0, s>>>(P, a1, omega, T, u, phi, a_new, A_al, A_ab, A_cp, A_Tp, AU[0],
                                                       AUl[0], partials, counter, grad);
  k_adj_adv_faces<1><<<grid_blocks(nv), BLOCK, 0, s>>>(P, a1, omega, T, v, phi, a_new, A_al, A_ab, A_cp, A_Tp, AU[1],
                                                       AUl[1], partials, counter, grad);
  k_adj_adv_faces<2><<<grid_blocks(nw), BLOCK, 0, s>>>(P, a1, omega, T, w, phi, a_new, A_al, A_ab, A_cp, A_Tp, AU[2],
                                                       AUl[2], partials, counter, grad);
  k_adj_adv_cells<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, a1, omega, T, u, v, w, phi, a_new, A_al, A_ab, A_cp, A_Tp,
                                                     A_a1, A_om, A_T, A_c);
}
void launch_adj_phi_rhs(const DevParams& P, double* const AUl[3], double* b, hipStream_t s) {
  k_adj_phi_rhs<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, AUl[0], AUl[1], AUl[2], b);
}
void launch_adj_phi_faces(const DevParams& P, double* const AUl[3], const double* lam, double* const AU[3],
                          hipStream_t s) {
  const long long nu = (long long)(P.nx + 1) * P.ny * P.nz, nv = (long long)P.nx * (P.ny + 1) * P.nz,
                  nw = (long long)P.nx * P.ny * (P.nz + 1);
  k_adj_phi_faces<0><<<grid_blocks(nu), BLOCK, 0, s>>>(P, AUl[0], lam, AU[0]);
  k_adj_phi_faces<1><<<grid_blocks(nv), BLOCK, 0, s>>>(P, AUl[1], lam, AU[1]);
  k_adj_phi_faces<2><<<grid_blocks(nw), BLOCK, 0, s>>>(P, AUl[2], lam, AU[2]);
}
void launch_adj_source(const DevParams& P, const double* alpha, const double* mraw, const double* A_a1, double* A_md,
                       double* A_al, const double* scal, double* partials, unsigned* counter, double* grad,
                       hipStream_t s) {
  k_adj_source<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, alpha, mraw, A_a1, A_md, A_al, scal, partials, counter, grad);
}
void launch_adj_interface(const DevParams& P, const double* alpha, const double* T, const double* omega,
                          const double* u, const double* v, const double* w, const double* mraw, const int* adj,
                          const double* A_md, const double* scal, double* A_al, double* A_T, double* A_om,
                          double* const AU[3], const IfaceRecords& R, double* partials, unsigned* counter,
                          double* grad, hipStream_t s) {
  const int nb = grid_blocks(P.n);
  k_adj_iface_clear<<<nb, BLOCK, 0, s>>>(P, R);
  k_adj_interface<<<nb, BLOCK, 0, s>>>(P, alpha, T, omega, u, v, w, mraw, adj, A_md, scal, A_al, A_T, R, partials,
                                       counter, grad);
  k_adj_iface_gather<<<nb, BLOCK, 0, s>>>(P, adj, R, A_al);
  k_adj_iface_targets<<<nb, BLOCK, 0, s>>>(P, adj, R, A_om);
  k_adj_iface_faces<<<nb, BLOCK, 0, s>>>(P, R, AU[0], AU[1], AU[2]);
}
void launch_adj_init_c(const DevParams& P, const double* alpha, const double* omega, const double* A_c, double* A_al,
                       double* A_om, double* partials, unsigned* counter, double* grad, hipStream_t s) {
  k_adj_init_c<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, alpha, omega, A_c, A_al, A_om, partials, counter, grad);
}

}  // namespace dsv
