// Matrix-free Jacobi-preconditioned conjugate gradients for the symmetric
// positive definite 7-point systems of the step (implicit Euler of eqs. 7-9).
//
// Operator: (A x)_c = diag_c x_c - sum_{interior nb} sc (q_c + q_nb)/2 x_nb,
// with diag holding the Helmholtz term, the face sum and Dirichlet boundary
// coefficients.  Dot products are FP64 block partials combined in a fixed
// order by the last block (deterministic).  Every kernel first reads the
// device-side status and returns at once when the solve has finished, so the
// host can enqueue iterations in batches and test convergence once a batch.
#include <hip/hip_runtime.h>

#include "ds_device.h"
#include "ds_kernels.h"

namespace dsv {

__device__ __forceinline__ double apply_row(const DevParams& P, double sc, const double* __restrict__ qc,
                                            const double* __restrict__ diag, const double* __restrict__ x,
                                            long long c) {
  int i, j, k;
  decode(P, c, i, j, k);
  const double q = qc[c];
  const long long sx = (long long)P.ny * P.nz, sy = P.nz;
  double off = 0.0;
  if (i > 0) off += (q + qc[c - sx]) * x[c - sx];
  if (i < P.nx - 1) off += (q + qc[c + sx]) * x[c + sx];
  if (j > 0) off += (q + qc[c - sy]) * x[c - sy];
  if (j < P.ny - 1) off += (q + qc[c + sy]) * x[c + sy];
  if (k > 0) off += (q + qc[c - 1]) * x[c - 1];
  if (k < P.nz - 1) off += (q + qc[c + 1]) * x[c + 1];
  return diag[c] * x[c] - 0.5 * sc * off;
}

__global__ void k_pcg_init(DevParams P, double sc, const double* __restrict__ qc, const double* __restrict__ diag,
                           const double* __restrict__ b, const double* __restrict__ x, double* __restrict__ r,
                           double* __restrict__ pdir, SolveStatus* st, double* partials, unsigned* counter) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  double acc[3] = {0.0, 0.0, 0.0};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    const double bc = b[c];
    const double rc = bc - apply_row(P, sc, qc, diag, x, c);
    const double z = rc / diag[c];
    r[c] = rc;
    pdir[c] = z;
    acc[0] += bc * bc;
    acc[1] += rc * rc;
    acc[2] += rc * z;
  }
  const int ops[3] = {RSUM, RSUM, RSUM};
  if (block_reduce_publish<3>(acc, ops, partials, counter)) {
    double t[3];
    block_combine<3>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      st->bb = t[0];
      st->rr = t[1];
      st->bnorm = sqrt(t[0]);
      st->rz = t[2];
      st->it = 0;
      st->zero = t[0] == 0.0;
      st->res = t[0] == 0.0 ? 0.0 : sqrt(t[1]) / st->bnorm;
      st->done = (t[0] == 0.0 || st->res <= st->tol) ? 1 : 0;
    }
  }
}

__global__ void k_pcg_spmv(DevParams P, double sc, const double* __restrict__ qc, const double* __restrict__ diag,
                           const double* __restrict__ pdir, double* __restrict__ q, SolveStatus* st,
                           double* partials, unsigned* counter) {
  if (st->done) return;
  long long b0, b1;
  block_range(P.n, b0, b1);
  double acc[1] = {0.0};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    const double y = apply_row(P, sc, qc, diag, pdir, c);
    q[c] = y;
    acc[0] += pdir[c] * y;
  }
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double t[1];
    block_combine<1>(ops, partials, counter, t);
    if (threadIdx.x == 0) st->alpha = st->rz / t[0];
  }
}

__global__ void k_pcg_update(DevParams P, const double* __restrict__ diag, double* __restrict__ x,
                             double* __restrict__ r, const double* __restrict__ pdir,
                             const double* __restrict__ q, SolveStatus* st, double* partials,
                             unsigned* counter) {
  if (st->done) return;
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double a = st->alpha;
  double acc[2] = {0.0, 0.0};
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    x[c] += a * pdir[c];
    const double rc = r[c] - a * q[c];
    r[c] = rc;
    acc[0] += rc * rc;
    acc[1] += rc * (rc / diag[c]);
  }
  const int ops[2] = {RSUM, RSUM};
  if (block_reduce_publish<2>(acc, ops, partials, counter)) {
    double t[2];
    block_combine<2>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      st->it += 1;
      st->rr = t[0];
      st->res = sqrt(t[0]) / st->bnorm;
      if (st->res <= st->tol) {
        st->done = 1;
      } else if (st->it >= st->maxit) {
        st->done = 2;
      } else {
        st->beta = t[1] / st->rz;
        st->rz = t[1];
      }
    }
  }
}

__global__ void k_pcg_dir(DevParams P, const double* __restrict__ diag, const double* __restrict__ r,
                          double* __restrict__ pdir, const SolveStatus* st) {
  if (st->done) return;
  long long b0, b1;
  block_range(P.n, b0, b1);
  const double be = st->beta;
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) pdir[c] = r[c] / diag[c] + be * pdir[c];
}

__global__ void k_zero_if_flagged(double* x, long long n, const SolveStatus* st) {
  if (!st->zero) return;
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) x[c] = 0.0;
}

void launch_pcg_init(const DevParams& P, double sc, const double* qc, const double* diag,
                     const double* b, const double* x, double* r, double* pdir, SolveStatus* st,
                     double* partials, unsigned* counter, hipStream_t s) {
  k_pcg_init<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, sc, qc, diag, b, x, r, pdir, st, partials, counter);
}

void launch_pcg_iter(const DevParams& P, double sc, const double* qc, const double* diag,
                     double* x, double* r, double* pdir, double* q, SolveStatus* st,
                     double* partials, unsigned* counters, hipStream_t s) {
  const int nb = grid_blocks(P.n);
  k_pcg_spmv<<<nb, BLOCK, 0, s>>>(P, sc, qc, diag, pdir, q, st, partials, counters);
  k_pcg_update<<<nb, BLOCK, 0, s>>>(P, diag, x, r, pdir, q, st, partials, counters + 1);
  k_pcg_dir<<<nb, BLOCK, 0, s>>>(P, diag, r, pdir, st);
}

void launch_zero_if_flagged(double* x, long long n, const SolveStatus* st, hipStream_t s) {
  k_zero_if_flagged<<<grid_blocks(n), BLOCK, 0, s>>>(x, n, st);
}

}  // namespace dsv
