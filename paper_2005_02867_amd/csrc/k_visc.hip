// Implicit viscous momentum (eq. 5 / eq. 30: div mu (grad v + grad v^T), mu
// mixed by eq. 31).  After the inviscid predictor u*, each face component a
// solves on its interior faces
//   (rho_f/dt) u_a** - div(mu grad u_a**) = (rho_f/dt) u_a* + sum_b d_b(mu d_a u_b^n)
// (the transpose part explicit from the start-of-step velocities), with
// rho_f = 1/(1/rho)_f.  Fluxes along a sit in the cells (mu of the cell),
// across b != a on the edges (mean mu of the four cells around the edge, of
// the two inside the box on a boundary edge).  Box faces normal to a keep
// the predictor's values and enter as known neighbours; across walls and the
// forced inlet the tangential velocity is held at zero by a ghost -u half a
// cell outside (coefficient 2 mu_e/h^2), across open faces its gradient is
// zero.  The three components form one block-diagonal SPD system on the
// concatenated face vector [u | v | w], solved by Jacobi-preconditioned
// conjugate gradients with FP64 reductions; coefficients are formed on the
// fly from alpha'.
#include <hip/hip_runtime.h>

#include "ds_device.h"
#include "ds_kernels.h"

namespace dsv {

namespace {

struct Face {
  int a;          // component (normal axis)
  int i, j, k;    // indices in that component's face array
  long long loc;  // index within the component
};

__device__ __forceinline__ Face face_of(const DevParams& P, long long f, long long nu, long long nv) {
  Face F;
  if (f < nu) {
    F.a = 0;
    F.loc = f;
    decode3(f, P.ny, P.nz, F.i, F.j, F.k);
  } else if (f < nu + nv) {
    F.a = 1;
    F.loc = f - nu;
    decode3(F.loc, P.ny + 1, P.nz, F.i, F.j, F.k);
  } else {
    F.a = 2;
    F.loc = f - nu - nv;
    decode3(F.loc, P.ny, P.nz + 1, F.i, F.j, F.k);
  }
  return F;
}

__device__ __forceinline__ int ext(const DevParams& P, int ax) { return ax == 0 ? P.nx : (ax == 1 ? P.ny : P.nz); }

// Stride of axis ax in the face array of component a.
__device__ __forceinline__ long long fstride(const DevParams& P, int a, int ax) {
  const long long fy = P.ny + (a == 1), fz = P.nz + (a == 2);
  return ax == 0 ? fy * fz : (ax == 1 ? fz : 1);
}

__device__ __forceinline__ double mu_of(const DevParams& P, const double* alpha, int i, int j, int k) {
  const double ab = clamp01(alpha[cidx(P, i, j, k)]);
  return mix(ab, P.mu_L, P.mu_G);
}

// Coefficients of the row of interior face F: diagonal part m = rho_f/dt,
// K[2 ax + side] toward the neighbour across axis ax (side 0 low, 1 high),
// nb[2 ax + side]: that neighbour's offset in the component (0: none -- a
// ghost, its coefficient is in the diagonal, or a zero-gradient face),
// known[side]: the neighbour along a is a box face (a known value).
struct Row {
  double m, diag;
  double K[6];
  long long nb[6];
  bool known[2];
};

__device__ Row row_of(const DevParams& P, const double* alpha, const Face& F) {
  Row R;
  const double ih2 = 1.0 / (P.h * P.h);
  int c[3] = {F.i, F.j, F.k};
  const int a = F.a;
  int cl[3] = {c[0], c[1], c[2]}, cr[3] = {c[0], c[1], c[2]};
  cl[a] -= 1;   // cells on the two sides of the face along a
  const long long el = cidx(P, cl[0], cl[1], cl[2]), er = cidx(P, cr[0], cr[1], cr[2]);
  const double rl = mix(clamp01(alpha[el]), P.rho_L, rho_gas(P, el));
  const double rr = mix(clamp01(alpha[er]), P.rho_L, rho_gas(P, er));
  R.m = 1.0 / (P.dt * (0.5 * (1.0 / rl + 1.0 / rr)));
  const double mul = mu_of(P, alpha, cl[0], cl[1], cl[2]), mur = mu_of(P, alpha, cr[0], cr[1], cr[2]);
  R.diag = R.m;
  // along a: cells, the neighbours are faces a-1 and a+1
  R.K[2 * a] = mul * ih2;
  R.K[2 * a + 1] = mur * ih2;
  const long long sa = fstride(P, a, a);
  R.known[0] = c[a] - 1 == 0;
  R.known[1] = c[a] + 1 == ext(P, a);
  R.nb[2 * a] = -sa;
  R.nb[2 * a + 1] = sa;
  R.diag += R.K[2 * a] + R.K[2 * a + 1];
  for (int b = 0; b < 3; ++b) {
    if (b == a) continue;
    const long long sb = fstride(P, a, b);
    for (int side = 0; side < 2; ++side) {
      const int nbj = c[b] + (side ? 1 : -1);   // the neighbouring row across b
      double K;
      long long nb = 0;
      if (nbj < 0 || nbj >= ext(P, b)) {
        const int kind = P.kind[b * 2 + side];
        if (kind == WALL || kind == INLET) K = 2.0 * 0.5 * (mul + mur) * ih2;   // no slip
        else K = 0.0;                                                        // zero gradient
      } else {
        int ql[3] = {cl[0], cl[1], cl[2]}, qr[3] = {cr[0], cr[1], cr[2]};
        ql[b] = nbj;
        qr[b] = nbj;
        const double me = 0.25 * (mul + mur + mu_of(P, alpha, ql[0], ql[1], ql[2]) + mu_of(P, alpha, qr[0], qr[1], qr[2]));
        K = me * ih2;
        nb = side ? sb : -sb;
      }
      R.K[2 * b + side] = K;
      R.nb[2 * b + side] = nb;
      R.diag += K;
    }
  }
  return R;
}

__device__ __forceinline__ bool is_box_face(const DevParams& P, const Face& F) {
  const int p = F.a == 0 ? F.i : (F.a == 1 ? F.j : F.k);
  return p == 0 || p == ext(P, F.a);
}

// A x for the interior face F (neighbours on the box faces along a count as 0).
__device__ double apply_row(const DevParams& P, const Row& R, const double* x, long long f, const Face& F) {
  double y = R.diag * x[f];
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    if (R.nb[q] == 0) continue;
    if (q / 2 == F.a && R.known[q & 1]) continue;
    y -= R.K[q] * x[f + R.nb[q]];
  }
  return y;
}

// sum_b d_b(mu d_a u_b) at the interior face F from the face velocities u, v, w.
__device__ double transpose_part(const DevParams& P, const double* alpha, const Face& F, const double* const U[3]) {
  const double ih = 1.0 / P.h;
  const int a = F.a;
  int c[3] = {F.i, F.j, F.k};
  int cl[3] = {c[0], c[1], c[2]}, cr[3] = {c[0], c[1], c[2]};
  cl[a] -= 1;
  const double mul = mu_of(P, alpha, cl[0], cl[1], cl[2]), mur = mu_of(P, alpha, cr[0], cr[1], cr[2]);
  // b = a: mu d_a u_a in the two cells
  const double* Ua = U[a];
  const long long sa = fstride(P, a, a);
  const long long e = ((long long)F.i * (P.ny + (a == 1)) + F.j) * (P.nz + (a == 2)) + F.k;
  double t = (mur * (Ua[e + sa] - Ua[e]) - mul * (Ua[e] - Ua[e - sa])) * ih * ih;
  for (int b = 0; b < 3; ++b) {
    if (b == a) continue;
    const double* Ub = U[b];
    double st[2];
    for (int side = 0; side < 2; ++side) {
      const int bf = c[b] + side;   // the b-face index of this edge
      // u_b on the two a-cells at that b-face
      int fl[3] = {cl[0], cl[1], cl[2]}, fr[3] = {cr[0], cr[1], cr[2]};
      fl[b] = bf;
      fr[b] = bf;
      const long long sy = P.ny + (b == 1), sz = P.nz + (b == 2);
      const double ul = Ub[((long long)fl[0] * sy + fl[1]) * sz + fl[2]];
      const double ur = Ub[((long long)fr[0] * sy + fr[1]) * sz + fr[2]];
      // mu on the edge: the cells on both sides across b, or the two inside the box
      double me;
      if (bf == 0 || bf == ext(P, b)) {
        me = 0.5 * (mul + mur);
      } else {
        const int other = side ? c[b] + 1 : c[b] - 1;
        int ql[3] = {cl[0], cl[1], cl[2]}, qr[3] = {cr[0], cr[1], cr[2]};
        ql[b] = other;
        qr[b] = other;
        me = 0.25 * (mul + mur + mu_of(P, alpha, ql[0], ql[1], ql[2]) + mu_of(P, alpha, qr[0], qr[1], qr[2]));
      }
      st[side] = me * (ur - ul) * ih;
    }
    t += (st[1] - st[0]) * ih;
  }
  return t;
}

struct VView {
  long long nu, nv, nf;
};

// x = u* (all faces), b = right-hand side and d = diagonal on interior faces
// (box faces: b = d = 0).
__global__ void __launch_bounds__(BLOCK) k_visc_setup(DevParams P, VView V, const double* __restrict__ alpha, const double* __restrict__ us,
                             const double* __restrict__ vs, const double* __restrict__ ws,
                             const double* __restrict__ u, const double* __restrict__ v,
                             const double* __restrict__ w, double* __restrict__ x, double* __restrict__ b,
                             double* __restrict__ d) {
  long long b0, b1;
  block_range(V.nf, b0, b1);
  const double* const S[3] = {us, vs, ws};
  const double* const U[3] = {u, v, w};
  for (long long f = b0 + threadIdx.x; f < b1; f += BLOCK) {
    const Face F = face_of(P, f, V.nu, V.nv);
    const double xs = S[F.a][F.loc];
    x[f] = xs;
    if (is_box_face(P, F)) {
      b[f] = 0.0;
      d[f] = 0.0;
      continue;
    }
    const Row R = row_of(P, alpha, F);
    double rhs = R.m * xs + transpose_part(P, alpha, F, U);
    const long long sa = fstride(P, F.a, F.a);
    if (R.known[0]) rhs += R.K[2 * F.a] * S[F.a][F.loc - sa];
    if (R.known[1]) rhs += R.K[2 * F.a + 1] * S[F.a][F.loc + sa];
    b[f] = rhs;
    d[f] = R.diag;
  }
}

// r = b - A x, p = r/d; <r, r/d>, <b, b>, <r, r> -> status.
__global__ void __launch_bounds__(BLOCK) k_visc_resid(DevParams P, VView V, const double* __restrict__ alpha, const double* __restrict__ x,
                             const double* __restrict__ b, const double* __restrict__ d, double* __restrict__ r,
                             double* __restrict__ p, SolveStatus* st, double* partials, unsigned* counter) {
  long long b0, b1;
  block_range(V.nf, b0, b1);
  double acc[3] = {0.0, 0.0, 0.0};
  for (long long f = b0 + threadIdx.x; f < b1; f += BLOCK) {
    const Face F = face_of(P, f, V.nu, V.nv);
    if (is_box_face(P, F)) {
      r[f] = 0.0;
      p[f] = 0.0;
      continue;
    }
    const Row R = row_of(P, alpha, F);
    const double rv = b[f] - apply_row(P, R, x, f, F);
    const double z = rv / d[f];
    r[f] = rv;
    p[f] = z;
    acc[0] += rv * z;
    acc[1] += b[f] * b[f];
    acc[2] += rv * rv;
  }
  const int ops[3] = {RSUM, RSUM, RSUM};
  if (block_reduce_publish<3>(acc, ops, partials, counter)) {
    double t[3];
    block_combine<3>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      st->rz = t[0];
      st->bb = t[1];
      st->bnorm = sqrt(t[1]);
      st->rr = t[2];
      st->it = 0;
      st->zero = t[1] == 0.0;
      st->res = t[1] == 0.0 ? 0.0 : sqrt(t[2]) / st->bnorm;
      st->done = (t[1] == 0.0 || st->res <= st->tol) ? 1 : 0;
    }
  }
}

// q = A p, <p, q> -> alpha = rz / <p, q>.
__global__ void __launch_bounds__(BLOCK) k_visc_apply(DevParams P, VView V, const double* __restrict__ alpha, const double* __restrict__ p,
                             double* __restrict__ q, SolveStatus* st, double* partials, unsigned* counter) {
  if (st->done) return;
  long long b0, b1;
  block_range(V.nf, b0, b1);
  double acc[1] = {0.0};
  for (long long f = b0 + threadIdx.x; f < b1; f += BLOCK) {
    const Face F = face_of(P, f, V.nu, V.nv);
    if (is_box_face(P, F)) {
      q[f] = 0.0;
      continue;
    }
    const Row R = row_of(P, alpha, F);
    const double qv = apply_row(P, R, p, f, F);
    q[f] = qv;
    acc[0] += p[f] * qv;
  }
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double t[1];
    block_combine<1>(ops, partials, counter, t);
    if (threadIdx.x == 0) st->alpha = t[0] > 0.0 ? st->rz / t[0] : 0.0;
  }
}

// x += alpha p, r -= alpha q; <r, r/d>, <r, r> -> beta, residual, convergence.
__global__ void __launch_bounds__(BLOCK) k_visc_update(VView V, double* __restrict__ x, double* __restrict__ r, const double* __restrict__ p,
                              const double* __restrict__ q, const double* __restrict__ d, SolveStatus* st,
                              double* partials, unsigned* counter) {
  if (st->done) return;
  long long b0, b1;
  block_range(V.nf, b0, b1);
  const double al = st->alpha;
  double acc[2] = {0.0, 0.0};
  for (long long f = b0 + threadIdx.x; f < b1; f += BLOCK) {
    const double dv = d[f];
    if (dv == 0.0) continue;   // box face
    x[f] += al * p[f];
    const double rv = r[f] - al * q[f];
    r[f] = rv;
    acc[0] += rv * rv / dv;
    acc[1] += rv * rv;
  }
  const int ops[2] = {RSUM, RSUM};
  if (block_reduce_publish<2>(acc, ops, partials, counter)) {
    double t[2];
    block_combine<2>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      st->beta = st->rz != 0.0 ? t[0] / st->rz : 0.0;
      st->rz = t[0];
      st->rr = t[1];
      st->it += 1;
      st->res = sqrt(t[1]) / st->bnorm;
      st->done = st->res <= st->tol ? 1 : (st->it >= st->maxit ? 2 : 0);
    }
  }
}

// p = r/d + beta p (interior faces).
__global__ void __launch_bounds__(BLOCK) k_visc_dir(VView V, const double* __restrict__ r, const double* __restrict__ d,
                           double* __restrict__ p, const SolveStatus* st) {
  if (st->done) return;
  long long b0, b1;
  block_range(V.nf, b0, b1);
  const double be = st->beta;
  for (long long f = b0 + threadIdx.x; f < b1; f += BLOCK) {
    const double dv = d[f];
    if (dv == 0.0) continue;
    p[f] = r[f] / dv + be * p[f];
  }
}

// u**, v**, w** on the interior faces from x.
__global__ void __launch_bounds__(BLOCK) k_visc_store(DevParams P, VView V, const double* __restrict__ x, double* __restrict__ us,
                             double* __restrict__ vs, double* __restrict__ ws) {
  long long b0, b1;
  block_range(V.nf, b0, b1);
  double* const S[3] = {us, vs, ws};
  for (long long f = b0 + threadIdx.x; f < b1; f += BLOCK) {
    const Face F = face_of(P, f, V.nu, V.nv);
    if (!is_box_face(P, F)) S[F.a][F.loc] = x[f];
  }
}

VView view_of(const DevParams& P) {
  VView V;
  V.nu = (long long)(P.nx + 1) * P.ny * P.nz;
  V.nv = (long long)P.nx * (P.ny + 1) * P.nz;
  V.nf = V.nu + V.nv + (long long)P.nx * P.ny * (P.nz + 1);
  return V;
}

}  // namespace

long long visc_faces(const DevParams& P) { return view_of(P).nf; }

void launch_visc_start(const DevParams& P, const double* a_new, const double* us, const double* vs, const double* ws,
                       const double* u, const double* v, const double* w, const ViscVecs& X, SolveStatus* st,
                       double* partials, unsigned* counter, hipStream_t s) {
  const VView V = view_of(P);
  const int nb = grid_blocks(V.nf);
  k_visc_setup<<<nb, BLOCK, 0, s>>>(P, V, a_new, us, vs, ws, u, v, w, X.x, X.b, X.d);
  k_visc_resid<<<nb, BLOCK, 0, s>>>(P, V, a_new, X.x, X.b, X.d, X.r, X.p, st, partials, counter);
}

void launch_visc_iteration(const DevParams& P, const double* a_new, const ViscVecs& X, SolveStatus* st,
                           double* partials, unsigned* counter, hipStream_t s) {
  const VView V = view_of(P);
  const int nb = grid_blocks(V.nf);
  k_visc_apply<<<nb, BLOCK, 0, s>>>(P, V, a_new, X.p, X.q, st, partials, counter);
  k_visc_update<<<nb, BLOCK, 0, s>>>(V, X.x, X.r, X.p, X.q, X.d, st, partials, counter);
  k_visc_dir<<<nb, BLOCK, 0, s>>>(V, X.r, X.d, X.p, st);
}

void launch_visc_store(const DevParams& P, const ViscVecs& X, double* us, double* vs, double* ws, hipStream_t s) {
  const VView V = view_of(P);
  k_visc_store<<<grid_blocks(V.nf), BLOCK, 0, s>>>(P, V, X.x, us, vs, ws);
}

}  // namespace dsv
