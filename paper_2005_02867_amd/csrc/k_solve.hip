// Matrix-free preconditioned conjugate gradients for the symmetric positive
// definite 7-point systems of the step (implicit Euler of eqs. 7-9):
//   (A x)_c = diag_c x_c - sc/2 sum_{interior nb} (q_c + q_nb) x_nb,
// diag holding the Helmholtz term, the face sum and the Dirichlet boundary
// coefficients.  Preconditioners: Jacobi (energy, species) or a geometric
// multigrid V-cycle (pressure).
//
// Multigrid: every level carries the same operator form, q averaged over the
// (up to 8) children of a coarse cell, sc = dt/H^2 on a level of spacing H,
// p_rgh = 0 box faces adding 2 sc q_c to the diagonal; restriction P^T/8,
// piecewise-constant prolongation, damped Jacobi with equal pre/post sweep
// counts, so the V-cycle is a symmetric positive definite preconditioner.
//
// Kernels are templated on the vector type (double, or float for the FP32
// inner solves of the mixed-precision form); dot products always accumulate
// in FP64, combined in a fixed order (deterministic).  Each kernel reads the
// device-side status first and returns when the solve has finished, so the
// host enqueues iterations in batches and tests convergence once per batch.
//
// Work decomposition: 64 (z) x 4 (y) cell tiles, one cell per thread, no
// integer division per cell.  XCD x (blocks are dealt to the 8 XCDs
// round-robin) owns one contiguous eighth of the tiles, i.e. a slab of
// x-planes, so stencil neighbours are served from that XCD's L2.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ds_device.h"
#include "ds_kernels.h"
#include "ds_mg.h"

namespace dsv {

__device__ __forceinline__ void tile_span(unsigned ntiles, unsigned& t0, unsigned& t1, unsigned& step) {
  const unsigned nb = gridDim.x, per = nb / NXCD, xcd = blockIdx.x % NXCD, local = blockIdx.x / NXCD;
  const unsigned chunk = (ntiles + NXCD - 1) / NXCD;
  t0 = xcd * chunk + local;
  t1 = min((xcd + 1) * chunk, ntiles);
  step = per;
}

template <class T>
__device__ __forceinline__ bool tile_cell(const Lev<T>& L, unsigned t, int& i, int& j, int& k, long long& c) {
  const unsigned kt = t % (unsigned)L.ntk;
  const unsigned r = t / (unsigned)L.ntk;
  const unsigned jt = r % (unsigned)L.ntj;
  i = (int)(r / (unsigned)L.ntj);
  k = (int)kt * TK + (int)(threadIdx.x & (TK - 1));
  j = (int)jt * TJ + (int)(threadIdx.x / TK);
  c = ((long long)i * L.ny + j) * L.nz + k;
  return j < L.ny && k < L.nz;
}

static int tile_blocks(unsigned ntiles) {
  unsigned nb = std::min<unsigned>(std::max<unsigned>(ntiles, NXCD), MAX_BLOCKS);
  return (int)((nb + NXCD - 1) / NXCD * NXCD);
}

// Loop over this block's cells: declares i, j, k (cell) and c (flat index).
#define FOR_CELLS(L, i, j, k, c)               \
  unsigned t0_, t1_, st_;                      \
  tile_span((L).ntiles, t0_, t1_, st_);        \
  int i, j, k;                                 \
  long long c;                                 \
  for (unsigned t_ = t0_; t_ < t1_; t_ += st_) \
    if (tile_cell(L, t_, i, j, k, c))

// Off-diagonal sum_nb (q_c + q_nb) x_nb, with the neighbour values given by xf(offset).
template <class T, class F>
__device__ __forceinline__ T off_sum(const Lev<T>& L, long long c, int i, int j, int k, F xf) {
  const T q = L.qc[c];
  const long long sx = (long long)L.ny * L.nz, sy = L.nz;
  T off = 0;
  if (i > 0) off += (q + L.qc[c - sx]) * xf(c - sx);
  if (i < L.nx - 1) off += (q + L.qc[c + sx]) * xf(c + sx);
  if (j > 0) off += (q + L.qc[c - sy]) * xf(c - sy);
  if (j < L.ny - 1) off += (q + L.qc[c + sy]) * xf(c + sy);
  if (k > 0) off += (q + L.qc[c - 1]) * xf(c - 1);
  if (k < L.nz - 1) off += (q + L.qc[c + 1]) * xf(c + 1);
  return off;
}

template <class T>
__device__ __forceinline__ T apply_at(const Lev<T>& L, const T* __restrict__ x, long long c, int i, int j, int k) {
  return L.diag[c] * x[c] - T(0.5) * L.sc * off_sum(L, c, i, j, k, [&](long long f) { return x[f]; });
}

// ------------------------------------------------------------ multigrid setup
template <class T>
__global__ void k_mg_coarsen_q(Lev<T> F, Lev<T> C, T* __restrict__ qout) {
  FOR_CELLS(C, I, J, K, c) {
    double s = 0.0;
    int cnt = 0;
    for (int di = 0; di < 2; ++di)
      for (int dj = 0; dj < 2; ++dj)
        for (int dk = 0; dk < 2; ++dk) {
          const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
          if (i < F.nx && j < F.ny && k < F.nz) {
            s += (double)F.qc[((long long)i * F.ny + j) * F.nz + k];
            ++cnt;
          }
        }
    qout[c] = (T)(s / cnt);
  }
}

template <class T>
__global__ void k_mg_diag(Lev<T> L, int dirmask, T* __restrict__ dout) {
  FOR_CELLS(L, i, j, k, c) {
    const double q = (double)L.qc[c], sc = (double)L.sc;
    const long long sx = (long long)L.ny * L.nz, sy = L.nz;
    double d = 0.0;
    if (i > 0) d += sc * 0.5 * (q + (double)L.qc[c - sx]); else if (dirmask & 1) d += 2.0 * sc * q;
    if (i < L.nx - 1) d += sc * 0.5 * (q + (double)L.qc[c + sx]); else if (dirmask & 2) d += 2.0 * sc * q;
    if (j > 0) d += sc * 0.5 * (q + (double)L.qc[c - sy]); else if (dirmask & 4) d += 2.0 * sc * q;
    if (j < L.ny - 1) d += sc * 0.5 * (q + (double)L.qc[c + sy]); else if (dirmask & 8) d += 2.0 * sc * q;
    if (k > 0) d += sc * 0.5 * (q + (double)L.qc[c - 1]); else if (dirmask & 16) d += 2.0 * sc * q;
    if (k < L.nz - 1) d += sc * 0.5 * (q + (double)L.qc[c + 1]); else if (dirmask & 32) d += 2.0 * sc * q;
    dout[c] = (T)d;
  }
}

// ------------------------------------------------------------ V-cycle pieces
template <class T>
__global__ void k_mg_smooth_zero(Lev<T> L, const T* __restrict__ r, T* __restrict__ x, T omega,
                                 const SolveStatus* st) {
  if (st->done) return;
  FOR_CELLS(L, i, j, k, c) { x[c] = omega * r[c] / L.diag[c]; }
}

// Publish <r, z> of the preconditioned residual: beta = rz_new/rz (unless first).
template <int NT = BLOCK>
__device__ __forceinline__ void publish_rz(double acc0, SolveStatus* st, double* partials, unsigned* counter,
                                           int first) {
  double acc[1] = {acc0};
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1, NT>(acc, ops, partials, counter)) {
    double t[1];
    block_combine<1, NT>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      if (!first) st->beta = t[0] / st->rz;
      st->rz = t[0];
    }
  }
}

// x_out = x_in + omega (r - A x_in)/diag; with DOT, also <r, x_out>.
template <class T, bool DOT>
__global__ void k_mg_smooth(Lev<T> L, const T* __restrict__ r, const T* __restrict__ xin, T* __restrict__ xout,
                            T omega, SolveStatus* st, double* partials, unsigned* counter, int first) {
  if (st->done) return;
  double acc = 0.0;
  FOR_CELLS(L, i, j, k, c) {
    const T rc = r[c];
    const T xn = xin[c] + omega * (rc - apply_at(L, xin, c, i, j, k)) / L.diag[c];
    xout[c] = xn;
    if (DOT) acc += (double)rc * (double)xn;
  }
  if (DOT) publish_rz(acc, st, partials, counter, first);
}

// Coarse residual: rc[C] = (1/8) sum_children (r - A x).
template <class T>
__global__ void k_mg_restrict(Lev<T> F, Lev<T> C, const T* __restrict__ r, const T* __restrict__ x,
                              T* __restrict__ rc, const SolveStatus* st) {
  if (st->done) return;
  FOR_CELLS(C, I, J, K, cc) {
    T s = 0;
    for (int di = 0; di < 2; ++di)
      for (int dj = 0; dj < 2; ++dj)
        for (int dk = 0; dk < 2; ++dk) {
          const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
          if (i < F.nx && j < F.ny && k < F.nz) {
            const long long f = ((long long)i * F.ny + j) * F.nz + k;
            s += r[f] - apply_at(F, x, f, i, j, k);
          }
        }
    rc[cc] = T(0.125) * s;
  }
}

// x' = x + P xc (piecewise constant), then one smoothing sweep on x'.
template <class T, bool DOT>
__global__ void k_mg_prolong_smooth(Lev<T> F, Lev<T> C, const T* __restrict__ r, const T* __restrict__ x,
                                    const T* __restrict__ xc, T* __restrict__ xout, T omega, SolveStatus* st,
                                    double* partials, unsigned* counter, int first) {
  if (st->done) return;
  double acc = 0.0;
  const long long sx = (long long)F.ny * F.nz, sy = F.nz;
  FOR_CELLS(F, i, j, k, c) {
    auto par = [&](int ii, int jj, int kk) -> long long {
      return ((long long)(ii >> 1) * C.ny + (jj >> 1)) * C.nz + (kk >> 1);
    };
    const T q = F.qc[c];
    T off = 0;
    if (i > 0) off += (q + F.qc[c - sx]) * (x[c - sx] + xc[par(i - 1, j, k)]);
    if (i < F.nx - 1) off += (q + F.qc[c + sx]) * (x[c + sx] + xc[par(i + 1, j, k)]);
    if (j > 0) off += (q + F.qc[c - sy]) * (x[c - sy] + xc[par(i, j - 1, k)]);
    if (j < F.ny - 1) off += (q + F.qc[c + sy]) * (x[c + sy] + xc[par(i, j + 1, k)]);
    if (k > 0) off += (q + F.qc[c - 1]) * (x[c - 1] + xc[par(i, j, k - 1)]);
    if (k < F.nz - 1) off += (q + F.qc[c + 1]) * (x[c + 1] + xc[par(i, j, k + 1)]);
    const long long pc = par(i, j, k);
    const T x0 = x[c] + xc[pc];
    const T rc = r[c];
    const T Ax = F.diag[c] * x0 - T(0.5) * F.sc * off;
    const T xn = x0 + omega * (rc - Ax) / F.diag[c];
    xout[c] = xn;
    if (DOT) acc += (double)rc * (double)xn;
  }
  if (DOT) publish_rz(acc, st, partials, counter, first);
}

// All sweeps of the coarsest level in one workgroup (the level fits in LDS):
// x = omega r/diag, then sweeps-1 damped-Jacobi sweeps, ping-pong in LDS;
// with DOT the last sweep also publishes <r, x>.  Replaces `sweeps` launches
// of a few microseconds each by one.
constexpr int COARSE_MAX = 1024;   // cells of a level solved this way
template <class T, bool DOT>
__global__ void __launch_bounds__(BLOCK) k_mg_coarse(Lev<T> L, const T* __restrict__ r, T* __restrict__ xout,
                                                     T omega, int sweeps, SolveStatus* st, double* partials,
                                                     unsigned* counter, int first) {
  if (st->done) return;
  __shared__ T sr[COARSE_MAX], sq[COARSE_MAX], sd[COARSE_MAX], xa[COARSE_MAX], xb[COARSE_MAX];
  const int n = (int)L.n;
  for (int c = threadIdx.x; c < n; c += BLOCK) {
    sr[c] = r[c];
    sq[c] = L.qc[c];
    sd[c] = L.diag[c];
    xa[c] = omega * sr[c] / sd[c];
  }
  __syncthreads();
  T* a = xa;
  T* b = xb;
  const int sx = L.ny * L.nz, sy = L.nz;
  double acc = 0.0;
  for (int t = 1; t < sweeps; ++t) {
    const bool last = t == sweeps - 1;
    for (int c = threadIdx.x; c < n; c += BLOCK) {
      const int k = c % L.nz, j = (c / L.nz) % L.ny, i = c / sx;
      const T q = sq[c];
      T off = 0;
      if (i > 0) off += (q + sq[c - sx]) * a[c - sx];
      if (i < L.nx - 1) off += (q + sq[c + sx]) * a[c + sx];
      if (j > 0) off += (q + sq[c - sy]) * a[c - sy];
      if (j < L.ny - 1) off += (q + sq[c + sy]) * a[c + sy];
      if (k > 0) off += (q + sq[c - 1]) * a[c - 1];
      if (k < L.nz - 1) off += (q + sq[c + 1]) * a[c + 1];
      const T ax = sd[c] * a[c] - T(0.5) * L.sc * off;
      const T xn = a[c] + omega * (sr[c] - ax) / sd[c];
      b[c] = xn;
      if (DOT && last) acc += (double)sr[c] * (double)xn;
    }
    __syncthreads();
    T* tmp = a;
    a = b;
    b = tmp;
  }
  for (int c = threadIdx.x; c < n; c += BLOCK) xout[c] = a[c];
  if (DOT) publish_rz(acc, st, partials, counter, first);
}

// ------------------------------------------------------------ CG pieces
__global__ void k_resid64(Lev<double> L, const double* __restrict__ b, const double* __restrict__ x,
                          double* __restrict__ r, SolveStatus* st, double* partials, unsigned* counter,
                          int set_bnorm) {
  double acc[2] = {0.0, 0.0};
  FOR_CELLS(L, i, j, k, c) {
    const double bc = b[c];
    const double rc = bc - apply_at(L, x, c, i, j, k);
    r[c] = rc;
    acc[0] += bc * bc;
    acc[1] += rc * rc;
  }
  const int ops[2] = {RSUM, RSUM};
  if (block_reduce_publish<2>(acc, ops, partials, counter)) {
    double t[2];
    block_combine<2>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      if (set_bnorm) {
        st->bb = t[0];
        st->bnorm = sqrt(t[0]);
        st->it = 0;
      }
      st->rr = t[1];
      st->zero = st->bb == 0.0;
      st->res = st->bb == 0.0 ? 0.0 : sqrt(t[1]) / st->bnorm;
      st->done = (st->bb == 0.0 || st->res <= st->tol) ? 1 : 0;
    }
  }
}

// Inner-solve start: r = (T) r64, x = 0; the inner reference norm is ||r||.
template <class T>
__global__ void k_inner_init(Lev<T> L, const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ x,
                             SolveStatus* st, double* partials, unsigned* counter) {
  double acc[1] = {0.0};
  FOR_CELLS(L, i, j, k, c) {
    const T v = (T)r64[c];
    r[c] = v;
    x[c] = 0;
    acc[0] += (double)v * (double)v;
  }
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double t[1];
    block_combine<1>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      st->bb = t[0];
      st->bnorm = sqrt(t[0]);
      st->rr = t[0];
      st->res = t[0] == 0.0 ? 0.0 : 1.0;
      st->it = 0;
      st->zero = t[0] == 0.0;
      st->done = t[0] == 0.0 ? 1 : 0;
    }
  }
}

// Jacobi start: rz = sum r^2/diag.
template <class T>
__global__ void k_jac_rz(Lev<T> L, const T* __restrict__ r, SolveStatus* st, double* partials, unsigned* counter,
                         int first) {
  if (st->done) return;
  double acc = 0.0;
  FOR_CELLS(L, i, j, k, c) {
    const double rc = (double)r[c];
    acc += rc * rc / (double)L.diag[c];
  }
  publish_rz(acc, st, partials, counter, first);
}

// p_out = z + beta p_in (z = r/diag for Jacobi), q = A p_out, <p, q> -> alpha.
template <class T, bool JAC>
__global__ void k_cg_dir_spmv(Lev<T> L, const T* __restrict__ z, const T* __restrict__ r, const T* __restrict__ pin,
                              T* __restrict__ pout, T* __restrict__ q, SolveStatus* st, double* partials,
                              unsigned* counter, int first) {
  if (st->done) return;
  const T be = first ? T(0) : (T)st->beta;
  double acc[1] = {0.0};
  FOR_CELLS(L, i, j, k, c) {
    auto pn = [&](long long f) -> T {
      const T zf = JAC ? r[f] / L.diag[f] : z[f];
      return first ? zf : zf + be * pin[f];
    };
    const T pc = pn(c);
    const T y = L.diag[c] * pc - T(0.5) * L.sc * off_sum(L, c, i, j, k, pn);
    pout[c] = pc;
    q[c] = y;
    acc[0] += (double)pc * (double)y;
  }
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double t[1];
    block_combine<1>(ops, partials, counter, t);
    if (threadIdx.x == 0) st->alpha = st->rz / t[0];
  }
}

// x += alpha p, r -= alpha q, ||r|| -> convergence; Jacobi: rz -> beta.
template <class T, bool JAC>
__global__ void k_cg_update(Lev<T> L, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                            const T* __restrict__ q, SolveStatus* st, double* partials, unsigned* counter) {
  if (st->done) return;
  const T a = (T)st->alpha;
  double acc[2] = {0.0, 0.0};
  FOR_CELLS(L, i, j, k, c) {
    x[c] += a * p[c];
    const T rc = r[c] - a * q[c];
    r[c] = rc;
    acc[0] += (double)rc * (double)rc;
    if (JAC) acc[1] += (double)rc * (double)rc / (double)L.diag[c];
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
      } else if (JAC) {
        st->beta = t[1] / st->rz;
        st->rz = t[1];
      }
    }
  }
}

template <class T>
__global__ void k_add_correction(Lev<T> L, double* __restrict__ x, const T* __restrict__ e) {
  FOR_CELLS(L, i, j, k, c) { x[c] += (double)e[c]; }
}

__global__ void k_to_float(const double* __restrict__ a, float* __restrict__ b, long long n) {
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) b[c] = (float)a[c];
}

// b = 0: the solution is x = 0, and its residual r = b - A 0 = 0 (r may be null).
__global__ void k_zero_if_flagged(double* x, double* r, long long n, const SolveStatus* st) {
  if (!st->zero) return;
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long c = b0 + threadIdx.x; c < b1; c += BLOCK) {
    x[c] = 0.0;
    if (r) r[c] = 0.0;
  }
}

// ------------------------------------------------------------ z-vectorised kernels
// Levels whose nz is a multiple of VW<T> (4 floats or 2 doubles, 16 bytes)
// run these variants: each thread owns VW consecutive z cells, loaded and
// stored as one 16-byte vector, so a wavefront moves 1 KiB per load
// instruction instead of 256 B (float).  Items (i, j, kv) are numbered
// z-fastest; each XCD streams one contiguous eighth of them.  The
// arithmetic and its order per cell are those of the scalar kernels above.
template <class T>
struct VW;
template <>
struct VW<float> {
  static constexpr int n = 4;
  typedef float4 vec;
};
template <>
struct VW<double> {
  static constexpr int n = 2;
  typedef double2 vec;
};

template <class T>
__device__ __forceinline__ void ldv(const T* __restrict__ p, T (&o)[VW<T>::n]) {
  const typename VW<T>::vec v = *reinterpret_cast<const typename VW<T>::vec*>(p);
  if constexpr (VW<T>::n == 4) {
    o[0] = v.x;
    o[1] = v.y;
    o[2] = v.z;
    o[3] = v.w;
  } else {
    o[0] = v.x;
    o[1] = v.y;
  }
}
template <class T>
__device__ __forceinline__ void stv(T* __restrict__ p, const T (&o)[VW<T>::n]) {
  typename VW<T>::vec v;
  if constexpr (VW<T>::n == 4) {
    v.x = o[0];
    v.y = o[1];
    v.z = o[2];
    v.w = o[3];
  } else {
    v.x = o[0];
    v.y = o[1];
  }
  *reinterpret_cast<typename VW<T>::vec*>(p) = v;
}
// Element e of an array through a 32-bit byte offset: loads and stores then
// take the scalar-base + 32-bit-offset form (one VGPR per address, shared by
// every array indexed alike).  use_vec() keeps each array below 4 GiB.
template <class T>
__device__ __forceinline__ T* at(T* p, unsigned e) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(p) + e * (unsigned)sizeof(T));
}
template <class T>
__device__ __forceinline__ const T* at(const T* p, unsigned e) {
  return reinterpret_cast<const T*>(reinterpret_cast<const char*>(p) + e * (unsigned)sizeof(T));
}

// The vectorised kernels run at most 1024 blocks of 4 waves, i.e. 4 waves per
// SIMD: the compiler may use up to 128 VGPRs and keep every load of an item
// in flight before the first wait.
#define VEC_KERNEL __global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(4, 4)))
// The marching kernels take their block size NT (256, 384 or 512 threads) as
// a template parameter, chosen per level so that a block holds whole z-rows
// (see march_lev): 384 fits rows of 24, 48, 96 or 192 vectors, 512 gives 256-
// cell FP32 rows eight rows per block.
#define VEC_KERNEL_M __global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(4, 4)))

// Vectorised kernels: nz a multiple of the vector width and every array
// (FP64 ones included) below 4 GiB, so 32-bit byte offsets address it.
template <class T>
inline bool use_vec(const Lev<T>& L) {
  return L.nz % VW<T>::n == 0 && L.n < (1LL << 29);
}
template <class T>
inline long long vec_items(const Lev<T>& L) {
  return (long long)L.nx * L.ny * (L.nz / VW<T>::n);
}
static const LaunchShape k_default_shape{};
static thread_local const LaunchShape* t_shape = nullptr;
const LaunchShape& launch_shape() { return t_shape ? *t_shape : k_default_shape; }
ShapeScope::ShapeScope(const LaunchShape* s) : prev_(t_shape) { t_shape = s; }
ShapeScope::~ShapeScope() { t_shape = prev_; }

void set_vec_max_blocks(LaunchShape& sh, int nb) {
  // every vectorised kernel publishes at most 2 partials per block
  nb = std::min(std::max(nb, NXCD), MAX_BLOCKS * MAX_RED / 2);
  sh.vec_max_blocks = nb / NXCD * NXCD;
}
static int vec_blocks(long long items) {
  long long nb = (items + BLOCK - 1) / BLOCK;
  nb = std::min<long long>(std::max<long long>(nb, NXCD), launch_shape().vec_max_blocks);
  return (int)((nb + NXCD - 1) / NXCD * NXCD);
}

// Loop over this block's items: declares i, j, kv and c (flat index of the first cell).
// Item order: kv fastest, then j within a slab of L.ytile rows, then i, then
// the slab.  Cell counts stay below 2^29 (use_vec), so items, cells and the
// decode all use 32-bit unsigned arithmetic.
#define FOR_ITEMS(L, T, i, j, kv, c)                                                                         \
  const int nzv_ = (L).nz / VW<T>::n;                                                                     \
  const unsigned nit_ = (unsigned)(L).nx * (unsigned)(L).ny * (unsigned)nzv_;                             \
  const unsigned per_ = gridDim.x / NXCD, loc_ = blockIdx.x / NXCD, xcd_ = blockIdx.x % NXCD;              \
  const unsigned yt_ = (unsigned)(L).ytile;                                                               \
  const unsigned chk_ = (nit_ + NXCD - 1) / NXCD;                                                         \
  const unsigned e0_ = xcd_ * chk_, e1_ = min(nit_, e0_ + chk_);                                          \
  int i, j, kv;                                                                                           \
  unsigned c;                                                                                             \
  unsigned t_, u_;                                                                                        \
  for (unsigned e_ = e0_ + loc_ * BLOCK + threadIdx.x; e_ < e1_; e_ += per_ * BLOCK)                      \
    if ((t_ = e_ / (unsigned)nzv_), (kv = (int)(e_ - t_ * (unsigned)nzv_)),                                 \
        (u_ = t_ / yt_), (j = (int)(t_ - u_ * yt_)), (i = (int)(u_ % (unsigned)(L).nx)),                     \
        (j += (int)(u_ / (unsigned)(L).nx * yt_)),                                                          \
        (c = ((unsigned)i * (unsigned)(L).ny + (unsigned)j) * (unsigned)(L).nz + (unsigned)kv * VW<T>::n), true)

// off[v] = sum_nb (q_v + q_nb) x_nb for the VW cells at c, in the scalar
// kernels' order (x-, x+, y-, y+, z-, z+).  xc: the cells' own x values;
// lx(f, out): vector of x at f; sx(f): scalar x at f.  The neighbour loads
// take no branch: a missing neighbour (domain edge) reads the cell itself and
// a select drops its term, so every load of the item is issued before the
// first wait instead of one neighbour's round trip after another.
template <class T, class LX, class SX>
__device__ __forceinline__ void off_sum_v(const Lev<T>& L, unsigned c, int i, int j, int kv, const T (&qv)[VW<T>::n],
                                          const T (&xc)[VW<T>::n], LX lx, SX sx, T (&off)[VW<T>::n]) {
  constexpr int V = VW<T>::n;
  const unsigned sxs = (unsigned)L.ny * (unsigned)L.nz, sys = (unsigned)L.nz;
  const int nzv = L.nz / V;
  const bool has[4] = {i > 0, i < L.nx - 1, j > 0, j < L.ny - 1};
  const unsigned f[4] = {has[0] ? c - sxs : c, has[1] ? c + sxs : c, has[2] ? c - sys : c, has[3] ? c + sys : c};
  const bool zm = kv > 0, zp = kv < nzv - 1;
  const unsigned fm = zm ? c - 1 : c, fp = zp ? c + V : c;
  T g[4][V], x[4][V];
#pragma unroll
  for (int n = 0; n < 4; ++n) {
    ldv<T>(at(L.qc, f[n]), g[n]);
    lx(f[n], x[n]);
  }
  const T gm = *at(L.qc, fm), xm = sx(fm), gp = *at(L.qc, fp), xp = sx(fp);
#pragma unroll
  for (int v = 0; v < V; ++v) off[v] = 0;
#pragma unroll
  for (int n = 0; n < 4; ++n)
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const T t = off[v] + (qv[v] + g[n][v]) * x[n][v];
      off[v] = has[n] ? t : off[v];
    }
  // z-: inside the vector, or the scalar before it
  {
    const T t = off[0] + (qv[0] + gm) * xm;
    off[0] = zm ? t : off[0];
  }
#pragma unroll
  for (int v = 1; v < V; ++v) off[v] += (qv[v] + qv[v - 1]) * xc[v - 1];
  // z+
#pragma unroll
  for (int v = 0; v < V - 1; ++v) off[v] += (qv[v] + qv[v + 1]) * xc[v + 1];
  {
    const T t = off[V - 1] + (qv[V - 1] + gp) * xp;
    off[V - 1] = zp ? t : off[V - 1];
  }
}

// ------------------------------------------------------- column marching
// The stencil kernels of the solvers walk the grid as columns: a thread owns
// one vector of VW cells of a y-z row, (j, kv), and steps through a chunk of
// x-planes.  q and the operand X of planes i-1, i, i+1 stay in registers
// across steps (the x neighbours cost no extra load), the z neighbours come
// from the adjacent lanes (lanes hold consecutive kv of a row; a load only at
// a wave's first and last lane), and only the y neighbours are loaded.
// Consecutive logical blocks run on one XCD, so the rows j-1, j+1 a block
// reads come from the same L2.

// Chunks per column: enough threads for about 1024 blocks of 256.
void set_march_threads(LaunchShape& sh, int n) { sh.march_threads = std::max(n, BLOCK); }
void set_march_min_planes(LaunchShape& sh, int n) { sh.march_min_planes = std::max(n, 1); }
// Block sizes tried in order, per kernel class (0: CG operator and FP64
// residual, 1: V-cycle sweeps and restriction); the first that holds whole
// z-rows of the level (every chunk's rows filling whole blocks) is taken,
// else 256 without row sharing.  Entries: 256, 384, 512; 0 ends the list.
void set_march_pref(LaunchShape& sh, int cls, const int* nts, int n) {
  if (cls < 0 || cls > 1) return;
  int k = 0;
  for (int t = 0; t < n && k < 3; ++t)
    if (nts[t] == 256 || nts[t] == 384 || nts[t] == 512) sh.march_pref[cls][k++] = nts[t];
  if (k == 0) sh.march_pref[cls][k++] = 256;
  for (; k < 4; ++k) sh.march_pref[cls][k] = 0;
}
// Block size of the level for class cls; pairs: also whole row pairs per
// block (the marching restriction).  0 when pairs is asked and none fits.
template <class T>
inline int march_nt(const Lev<T>& L, int cls, bool pairs) {
  const long long nzv = L.nz / VW<T>::n, rows = (long long)L.ny * nzv;
  const int* pref = launch_shape().march_pref[cls];
  for (int t = 0; t < 4 && pref[t]; ++t) {
    const int nt = pref[t];
    if (nt % nzv == 0 && rows % nt == 0 && (!pairs || ((nt / nzv) % 2 == 0))) return nt;
  }
  return pairs ? 0 : 256;
}
// threads: the thread count to aim for (0: the shape's march_threads).
template <class T>
inline Lev<T> march_lev(Lev<T> L, int cls = 0, long long threads = 0) {
  L.mnt = march_nt(L, cls, false);
  const long long ncol = (long long)L.ny * (L.nz / VW<T>::n);
  const LaunchShape& sh = launch_shape();
  const long long aim = threads > 0 ? threads : (long long)sh.march_threads;
  const long long nch = std::min<long long>(std::max<long long>((aim + ncol - 1) / ncol, 1), L.nx);
  const long long clen = std::max<long long>((L.nx + nch - 1) / nch, std::min(sh.march_min_planes, L.nx));
  L.mch = (int)((L.nx + clen - 1) / clen);   // no empty trailing chunks
  return L;
}
// Grid of the marching kernels: one thread per (column, chunk), at most
// 4096 blocks (threads then take several columns; every marching kernel
// publishes at most 2 partials per block).
template <class T>
inline int march_blocks(const Lev<T>& L) {
  const long long nt = (long long)L.ny * (L.nz / VW<T>::n) * L.mch;
  const long long nb = std::min<long long>(std::max<long long>((nt + L.mnt - 1) / L.mnt, NXCD), 4096);
  return (int)((nb + NXCD - 1) / NXCD * NXCD);
}

template <class T>
__device__ __forceinline__ T lane_up(T v) { return __shfl_up(v, 1, 64); }     // value of lane - 1
template <class T>
__device__ __forceinline__ T lane_down(T v) { return __shfl_down(v, 1, 64); } // value of lane + 1

// lx(f, out): operand vector at cell f; sx(f): operand at the single cell f;
// body(c, qc, xc, off, dg): the cells' own q and X, off = sum_nb (q + q_nb) X_nb
// (order x-, x+, y-, y+, z-, z+, as in the scalar kernels) and the diagonal.
// With L.dfly the diagonal is formed from the q values already in hand --
// sc (q + q_nb)/2 per neighbour, 2 sc q per Dirichlet box face, summed in FP64
// in face order as the setup kernels and k_mg_diag do -- instead of loaded.  Work items are
// (chunk, j, kv), kv fastest; a grid-stride loop covers them (the stride is a
// multiple of 64, so a wave's lanes always hold consecutive items).  Threads
// past the end do nothing and return normally (block reductions follow).
// ALT: odd chunks walk their planes downwards, so two neighbouring chunks
// read their shared boundary planes at the same step (the second read can
// come from the L2); the cell arithmetic is the same either way.  Kernels
// whose body depends on the walking order (the marching restriction) pass
// false.
// CQ: qc holds L.qk in every cell; q is taken from that value (no q loads or
// exchange), with the same arithmetic.
template <class T, int NT, bool ALT = true, bool CQ = false, class LX, class SX, class BODY>
__device__ __forceinline__ void march(const Lev<T>& L, LX lx, SX sx, BODY body) {
  constexpr int V = VW<T>::n;
  const T qk = L.qk;
  auto fillq = [&](T(&o)[V]) {
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = qk;
  };
  const unsigned nzv = (unsigned)L.nz / V, ny = (unsigned)L.ny, nx = (unsigned)L.nx;
  const unsigned nch = (unsigned)L.mch, clen = (nx + nch - 1) / nch;
  const unsigned per = gridDim.x / NXCD, lb = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  const unsigned total = ny * nzv * nch;
  const unsigned P = ny * (unsigned)L.nz, sy = (unsigned)L.nz;
  const int lane = threadIdx.x & 63;
  // Rows shared through LDS: when a block holds whole rows of one chunk
  // (nzv divides NT and every chunk's rows fill whole blocks), a thread's
  // y neighbours inside the block are the threads nzv before and after it;
  // each step they publish their (q, X) of the current plane in LDS (double
  // buffered by step parity, one barrier per step) and only the block's
  // first and last rows load their outer neighbour.  All threads of a block
  // then run the same steps, so the barriers are uniform.
  const bool coop = (NT % nzv == 0) && ((ny * nzv) % NT == 0);
  __shared__ T lsq[2][NT * V], lsx[2][NT * V];
  const int tid = threadIdx.x;
  const bool inm = coop && tid >= (int)nzv, inp = coop && tid + (int)nzv < NT;
  int par = 0;
  for (unsigned e = lb * NT + threadIdx.x; e < total; e += gridDim.x * NT) {
  const unsigned kv = e % nzv, t = e / nzv, j = t % ny, ch = t / ny;
  const unsigned i0 = ch * clen, i1 = min(nx, i0 + clen);
  if (i0 >= i1) continue;
  const bool hym = j > 0, hyp = j + 1 < ny, hzm = kv > 0, hzp = kv + 1 < nzv;
  const unsigned cj = j * sy + kv * V;
  const bool fw = !(ALT && (ch & 1u));
  const int dir = fw ? 1 : -1;
  const int sfirst = fw ? (int)i0 : (int)i1 - 1, slast = fw ? (int)i1 - 1 : (int)i0;
  auto clampp = [&](int q) { return q < 0 ? 0 : (q >= (int)nx ? (int)nx - 1 : q); };
  // qp, xp: the plane behind (walking direction); qc, xc: the current one
  T qp[V], xp[V], qc[V], xc[V];
  {
    const unsigned f = (unsigned)clampp(sfirst - dir) * P + cj;
    if (CQ) fillq(qp);
    else ldv<T>(at(L.qc, f), qp);
    lx(f, xp);
  }
  {
    const unsigned f = (unsigned)sfirst * P + cj;
    if (CQ) fillq(qc);
    else ldv<T>(at(L.qc, f), qc);
    lx(f, xc);
  }
  for (int i = sfirst;; i += dir) {
    const unsigned c = (unsigned)i * P + cj;
    const bool hxm = i > 0, hxp = i + 1 < (int)nx;
    const unsigned fn = (unsigned)clampp(i + dir) * P + cj, fym = hym ? c - sy : c, fyp = hyp ? c + sy : c;
    // qn, xn: the plane ahead
    T qn[V], xn[V], qym[V], xym[V], qyp[V], xyp[V];
    if (CQ) fillq(qn);
    else ldv<T>(at(L.qc, fn), qn);
    lx(fn, xn);
    if (!inm) {
      if (!CQ) ldv<T>(at(L.qc, fym), qym);
      lx(fym, xym);
    }
    if (!inp) {
      if (!CQ) ldv<T>(at(L.qc, fyp), qyp);
      lx(fyp, xyp);
    }
    if (coop) {
      if (!CQ) stv<T>(&lsq[par][tid * V], qc);
      stv<T>(&lsx[par][tid * V], xc);
      __syncthreads();
      if (inm) {
        if (!CQ) ldv<T>(&lsq[par][(tid - (int)nzv) * V], qym);
        ldv<T>(&lsx[par][(tid - (int)nzv) * V], xym);
      }
      if (inp) {
        if (!CQ) ldv<T>(&lsq[par][(tid + (int)nzv) * V], qyp);
        ldv<T>(&lsx[par][(tid + (int)nzv) * V], xyp);
      }
      par ^= 1;
    }
    if (CQ) {
      fillq(qym);
      fillq(qyp);
    }
    T qzm = CQ ? qk : lane_up(qc[V - 1]), xzm = lane_up(xc[V - 1]);
    T qzp = CQ ? qk : lane_down(qc[0]), xzp = lane_down(xc[0]);
    if (hzm && lane == 0) {
      if (!CQ) qzm = *at(L.qc, c - 1);
      xzm = sx(c - 1);
    }
    if (hzp && lane == 63) {
      if (!CQ) qzp = *at(L.qc, c + V);
      xzp = sx(c + V);
    }
    T off[V];
#pragma unroll
    for (int v = 0; v < V; ++v) off[v] = 0;
    auto nbr = [&](const T (&g)[V], const T (&x)[V], bool has) {
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const T tt = off[v] + (qc[v] + g[v]) * x[v];
        off[v] = has ? tt : off[v];
      }
    };
    // x neighbours on the minus and plus sides
    T qxm[V], xxm[V], qxp[V], xxp[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      qxm[v] = fw ? qp[v] : qn[v];
      xxm[v] = fw ? xp[v] : xn[v];
      qxp[v] = fw ? qn[v] : qp[v];
      xxp[v] = fw ? xn[v] : xp[v];
    }
    nbr(qxm, xxm, hxm);
    nbr(qxp, xxp, hxp);
    nbr(qym, xym, hym);
    nbr(qyp, xyp, hyp);
    {
      const T tt = off[0] + (qc[0] + qzm) * xzm;
      off[0] = hzm ? tt : off[0];
    }
#pragma unroll
    for (int v = 1; v < V; ++v) off[v] += (qc[v] + qc[v - 1]) * xc[v - 1];
#pragma unroll
    for (int v = 0; v < V - 1; ++v) off[v] += (qc[v] + qc[v + 1]) * xc[v + 1];
    {
      const T tt = off[V - 1] + (qc[V - 1] + qzp) * xzp;
      off[V - 1] = hzp ? tt : off[V - 1];
    }
    T dg[V];
    if (L.dfly) {
      const double sc = (double)L.sc;
      const int dm = L.dmask;
#pragma unroll
      for (int v = 0; v < V; ++v) {
        const double q = (double)qc[v], bnd = 2.0 * sc * q;
        double d = 0.0;
        d += hxm ? sc * 0.5 * (q + (double)qxm[v]) : ((dm & 1) ? bnd : 0.0);
        d += hxp ? sc * 0.5 * (q + (double)qxp[v]) : ((dm & 2) ? bnd : 0.0);
        d += hym ? sc * 0.5 * (q + (double)qym[v]) : ((dm & 4) ? bnd : 0.0);
        d += hyp ? sc * 0.5 * (q + (double)qyp[v]) : ((dm & 8) ? bnd : 0.0);
        const bool em = v > 0 || hzm, ep = v < V - 1 || hzp;
        const double gm = v > 0 ? (double)qc[v > 0 ? v - 1 : 0] : (double)qzm;
        const double gp = v < V - 1 ? (double)qc[v < V - 1 ? v + 1 : V - 1] : (double)qzp;
        d += em ? sc * 0.5 * (q + gm) : ((dm & 16) ? bnd : 0.0);
        d += ep ? sc * 0.5 * (q + gp) : ((dm & 32) ? bnd : 0.0);
        dg[v] = (T)d;
      }
    } else {
      ldv<T>(at(L.diag, c), dg);
    }
    body(c, qc, xc, off, dg);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      qp[v] = qc[v];
      xp[v] = xc[v];
      qc[v] = qn[v];
      xc[v] = xn[v];
    }
    if (i == slast) break;
  }
  }
}

template <class T>
__device__ __forceinline__ void apply_v(const Lev<T>& L, const T* __restrict__ x, unsigned c, int i, int j, int kv,
                                        const T (&xc)[VW<T>::n], T (&y)[VW<T>::n]) {
  constexpr int V = VW<T>::n;
  T qv[V], dg[V], off[V];
  ldv<T>(at(L.qc, c), qv);
  ldv<T>(at(L.diag, c), dg);
  off_sum_v<T>(L, c, i, j, kv, qv, xc, [&](unsigned f, T(&o)[V]) { ldv<T>(at(x, f), o); },
               [&](unsigned f) { return *at(x, f); }, off);
#pragma unroll
  for (int v = 0; v < V; ++v) y[v] = dg[v] * xc[v] - T(0.5) * L.sc * off[v];
}

template <class T>
VEC_KERNEL k_mg_smooth_zero_v(Lev<T> L, const T* __restrict__ r, T* __restrict__ x, T omega,
                                   const SolveStatus* st) {
  if (st->done) return;
  constexpr int V = VW<T>::n;
  FOR_ITEMS(L, T, i, j, kv, c) {
    T rv[V], dv[V], o[V];
    ldv<T>(at(r, c), rv);
    ldv<T>(at(L.diag, c), dv);
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = omega * rv[v] / dv[v];
    stv<T>(at(x, c), o);
  }
}

// The first two sweeps from x = 0 in one pass: x1 = omega r/diag is formed
// on the fly (also at the neighbours), x2 = x1 + omega (r - A x1)/diag.
template <class T, int NT>
VEC_KERNEL_M k_mg_smooth_two_v(Lev<T> L, const T* __restrict__ r, T* __restrict__ xout, T omega,
                                  const SolveStatus* st) {
  if (st->done) return;
  constexpr int V = VW<T>::n;
  auto x1v = [&](unsigned f, T(&o)[V]) {
    T rv[V], dv[V];
    ldv<T>(at(r, f), rv);
    ldv<T>(at(L.diag, f), dv);
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = omega * rv[v] / dv[v];
  };
  auto x1s = [&](unsigned f) -> T { return omega * *at(r, f) / *at(L.diag, f); };
  march<T, NT>(L, x1v, x1s, [&](unsigned c, const T(&qv)[V], const T(&x1)[V], const T(&off)[V], const T(&dv)[V]) {
    T rv[V], o[V];
    ldv<T>(at(r, c), rv);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const T ax = dv[v] * x1[v] - T(0.5) * L.sc * off[v];
      o[v] = x1[v] + omega * (rv[v] - ax) / dv[v];
    }
    stv<T>(at(xout, c), o);
  });
}

template <class T, bool DOT, int NT>
VEC_KERNEL_M k_mg_smooth_v(Lev<T> L, const T* __restrict__ r, const T* __restrict__ xin, T* __restrict__ xout,
                              T omega, SolveStatus* st, double* partials, unsigned* counter, int first) {
  if (st->done) return;
  constexpr int V = VW<T>::n;
  double acc = 0.0;
  march<T, NT>(
      L, [&](unsigned f, T(&o)[V]) { ldv<T>(at(xin, f), o); }, [&](unsigned f) { return *at(xin, f); },
      [&](unsigned c, const T(&qv)[V], const T(&xv)[V], const T(&off)[V], const T(&dv)[V]) {
        T rv[V], o[V];
        ldv<T>(at(r, c), rv);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const T ax = dv[v] * xv[v] - T(0.5) * L.sc * off[v];
          o[v] = xv[v] + omega * (rv[v] - ax) / dv[v];
          if (DOT) acc += (double)rv[v] * (double)o[v];
        }
        stv<T>(at(xout, c), o);
      });
  if (DOT) publish_rz<NT>(acc, st, partials, counter, first);
}

// Coarse residual for VW/2 coarse cells per thread (fine rows of VW cells).
template <class T>
VEC_KERNEL k_mg_restrict_v(Lev<T> F, Lev<T> C, const T* __restrict__ r, const T* __restrict__ x,
                                T* __restrict__ rc, const SolveStatus* st) {
  if (st->done) return;
  constexpr int V = VW<T>::n, H = V / 2;
  // items over the fine level's (I, J, kv) with I, J coarse rows: numbered as a
  // level of C.nx x C.ny x (F.nz / V) vector items
  Lev<T> G = C;
  G.nz = F.nz;   // kv ranges over F.nz / V
  FOR_ITEMS(G, T, I, J, kv, c_unused) {
    (void)c_unused;
    T s[H];
#pragma unroll
    for (int h = 0; h < H; ++h) s[h] = 0;
    for (int di = 0; di < 2; ++di)
      for (int dj = 0; dj < 2; ++dj) {
        const int i = 2 * I + di, j = 2 * J + dj;
        if (i >= F.nx || j >= F.ny) continue;
        const unsigned f = ((unsigned)i * (unsigned)F.ny + (unsigned)j) * (unsigned)F.nz + (unsigned)kv * V;
        T xv[V], rv[V], ax[V];
        ldv<T>(at(x, f), xv);
        ldv<T>(at(r, f), rv);
        apply_v<T>(F, x, f, i, j, kv, xv, ax);
#pragma unroll
        for (int h = 0; h < H; ++h) s[h] += (rv[2 * h] - ax[2 * h]) + (rv[2 * h + 1] - ax[2 * h + 1]);
      }
    const unsigned cc = ((unsigned)I * (unsigned)C.ny + (unsigned)J) * (unsigned)C.nz + (unsigned)kv * H;
#pragma unroll
    for (int h = 0; h < H; ++h) *at(rc, cc + h) = T(0.125) * s[h];
  }
}

// Coarse residual in marching form: the fine grid is walked as in the sweeps
// (so the fine residual r - A x costs the marching loads), each thread sums
// the residual pairs (2K, 2K+1) of its vector over the planes 2I, 2I+1, and
// the thread of row 2J+1 hands its sum through LDS to the thread of row 2J,
// which writes the coarse cell.  Needs even nx, ny, nz, chunks of an even
// number of planes and blocks of whole row pairs (restrict_marching_ok).
template <class T, int NT>
VEC_KERNEL_M k_mg_restrict_m(Lev<T> F, Lev<T> C, const T* __restrict__ r, const T* __restrict__ x,
                           T* __restrict__ rc, const SolveStatus* st) {
  if (st->done) return;
  constexpr int V = VW<T>::n, H = V / 2;
  __shared__ T lsr[NT * H];
  const unsigned nzv = (unsigned)F.nz / V, P = (unsigned)F.ny * (unsigned)F.nz, sy = (unsigned)F.nz;
  const int tid = threadIdx.x;
  T acc[H];
  march<T, NT, false>(
      F, [&](unsigned f, T(&o)[V]) { ldv<T>(at(x, f), o); }, [&](unsigned f) { return *at(x, f); },
      [&](unsigned c, const T(&qv)[V], const T(&xv)[V], const T(&off)[V], const T(&dv)[V]) {
        T rv[V];
        ldv<T>(at(r, c), rv);
        const unsigned i = c / P, rem = c - i * P, j = rem / sy, kv = (rem - j * sy) / V;
#pragma unroll
        for (int h = 0; h < H; ++h) {
          const T a0 = rv[2 * h] - (dv[2 * h] * xv[2 * h] - T(0.5) * F.sc * off[2 * h]);
          const T a1 = rv[2 * h + 1] - (dv[2 * h + 1] * xv[2 * h + 1] - T(0.5) * F.sc * off[2 * h + 1]);
          acc[h] = (i & 1u) ? acc[h] + (a0 + a1) : (a0 + a1);
        }
        if (i & 1u) {
          if (j & 1u) {
#pragma unroll
            for (int h = 0; h < H; ++h) lsr[tid * H + h] = acc[h];
          }
          __syncthreads();
          if (!(j & 1u)) {
            const unsigned cc = ((i >> 1) * (unsigned)C.ny + (j >> 1)) * (unsigned)C.nz + kv * H;
#pragma unroll
            for (int h = 0; h < H; ++h) *at(rc, cc + h) = T(0.125) * (acc[h] + lsr[(tid + (int)nzv) * H + h]);
          }
          __syncthreads();
        }
      });
}

// The marching restriction applies: even extents, whole row pairs per block,
// and the row sharing of the marching kernels (see march()).
template <class T>
inline bool restrict_marching_ok(const Lev<T>& F) {
  if (!use_vec(F) || (F.nx & 1) || (F.ny & 1) || (F.nz % (2 * VW<T>::n))) return false;
  return march_nt(F, 1, true) != 0;
}
// march_lev with chunks of an even number of planes (plane pairs stay
// together) and a block size of whole row pairs.
template <class T>
inline Lev<T> march_lev_pairs(Lev<T> L) {
  L = march_lev(L, 1);
  L.mnt = march_nt(L, 1, true);
  long long clen = (L.nx + L.mch - 1) / L.mch;
  clen += clen & 1;
  L.mch = (int)((L.nx + clen - 1) / clen);
  return L;
}

// x' = x + P xc then one sweep (VW fine cells per thread).
template <class T, bool DOT, int NT>
VEC_KERNEL_M k_mg_prolong_smooth_v(Lev<T> F, Lev<T> C, const T* __restrict__ r, const T* __restrict__ x,
                                      const T* __restrict__ xc, T* __restrict__ xout, T omega, SolveStatus* st,
                                      double* partials, unsigned* counter, int first) {
  if (st->done) return;
  constexpr int V = VW<T>::n;
  double acc = 0.0;
  // x + P xc for the vector of VW fine cells starting at fine index f
  auto row = [&](unsigned f, T(&o)[V]) {
    const unsigned rr = f / (unsigned)F.nz;   // ii*ny + jj
    const unsigned kk = f - rr * (unsigned)F.nz;
    const unsigned jj = rr % (unsigned)F.ny, ii = rr / (unsigned)F.ny;
    const unsigned pb = ((ii >> 1) * (unsigned)C.ny + (jj >> 1)) * (unsigned)C.nz + (kk >> 1);
    ldv<T>(at(x, f), o);
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] += *at(xc, pb + (v >> 1));
  };
  auto one = [&](unsigned f) -> T {
    const unsigned rr = f / (unsigned)F.nz;
    const unsigned kk = f - rr * (unsigned)F.nz;
    const unsigned jj = rr % (unsigned)F.ny, ii = rr / (unsigned)F.ny;
    return *at(x, f) + *at(xc, ((ii >> 1) * (unsigned)C.ny + (jj >> 1)) * (unsigned)C.nz + (kk >> 1));
  };
  march<T, NT>(F, row, one, [&](unsigned c, const T(&qv)[V], const T(&x0)[V], const T(&off)[V], const T(&dv)[V]) {
    T rv[V], o[V];
    ldv<T>(at(r, c), rv);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      const T Ax = dv[v] * x0[v] - T(0.5) * F.sc * off[v];
      o[v] = x0[v] + omega * (rv[v] - Ax) / dv[v];
      if (DOT) acc += (double)rv[v] * (double)o[v];
    }
    stv<T>(at(xout, c), o);
  });
  if (DOT) publish_rz<NT>(acc, st, partials, counter, first);
}

// ---------------------------------------------------------------- coloured sweeps
// One sweep of a two-colour smoother whose colours alternate along x and z:
// colour A holds the cells with i + k + c0 even, colour B the others.  A
// cell's x and z neighbours have the other colour, its y neighbours its own.
// Colour A is relaxed from x0 with the damped-Jacobi formula (weight w), then
// colour B from colour A's new values; y neighbours enter with their old
// values (Jacobi coupling along y).  The pre-smoothing sweeps relax the even
// colour first (c0 = 0) and the post-smoothing sweeps the odd one (c0 = 1),
// the reverse order, which keeps the V-cycle a symmetric preconditioner.
//
// Marching form as in march(), with colour A one plane ahead of colour B:
// the step for plane s relaxes plane s in colour A and finishes plane s - 1
// in colour B, so one pass over x0, r and q does both colours.  A chunk
// [i0, i1) also relaxes colour A on its outer planes i0 - 1 and i1, which its
// first and last planes need.  The y-neighbour term sum (q + q_y) x0_y of a
// plane serves both colours (old values either way) and is kept from one
// step to the next.  Needs the rows shared through LDS (rb_marching_ok): a
// z neighbour is then in an adjacent lane or, at a wave's edge, in the
// adjacent thread of the same block.
// lx(f, o): x0 vector at cell f (X0 false: x0 = 0, nothing loaded);
// out(c, o, rv): the finished vector of plane s - 1 and its r.
// CQ: qc holds L.qk in every cell; q is taken from that value (no q loads,
// no q exchange through LDS or lanes), with the same arithmetic.
template <class T, int NT, bool X0, bool WE, bool CQ, class LX, class OUT>
__device__ __forceinline__ void march_rb(const Lev<T>& L, const T* __restrict__ r, T w, int c0, LX lx, OUT out) {
  constexpr int V = VW<T>::n;
  const unsigned nzv = (unsigned)L.nz / V, ny = (unsigned)L.ny, nx = (unsigned)L.nx;
  const unsigned nch = (unsigned)L.mch, clen = (nx + nch - 1) / nch;
  const unsigned per = gridDim.x / NXCD, lb = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  const unsigned total = ny * nzv * nch;
  const unsigned P = ny * (unsigned)L.nz, sy = (unsigned)L.nz;
  const int tid = threadIdx.x;
  // lsm (WE: z-rows that span or straddle waves): each thread's first and
  // last colour-A value of the previous plane, for the wave-edge lanes whose
  // z neighbours sit in the adjacent wave of the same block
  __shared__ T lsq[2][NT * V], lsx[2][X0 ? NT * V : 1], lsm[2][WE ? 2 * NT : 1];
  const bool inm = tid >= (int)nzv, inp = tid + (int)nzv < NT;
  const int lane = tid & 63;
  const T hs = T(0.5) * L.sc;
  const T qk = L.qk;
  int par = 0;
  auto zero = [](T(&o)[V]) {
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = 0;
  };
  auto copy = [](T(&o)[V], const T(&a)[V]) {
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = a[v];
  };
  auto fillq = [&](T(&o)[V]) {
#pragma unroll
    for (int v = 0; v < V; ++v) o[v] = qk;
  };
  // out-of-range planes are clamped to the nearest one (loads stay inside
  // the array; the terms they would feed are switched off)
  auto clampp = [&](int q) { return q < 0 ? 0 : (q >= (int)nx ? (int)nx - 1 : q); };
  for (unsigned e = lb * NT + tid; e < total; e += gridDim.x * NT) {
    const unsigned kv = e % nzv, t = e / nzv, j = t % ny, ch = t / ny;
    const unsigned i0 = ch * clen, i1 = min(nx, i0 + clen);
    if (i0 >= i1) continue;
    const bool hym = j > 0, hyp = j + 1 < ny, hzm = kv > 0, hzp = kv + 1 < nzv;
    const unsigned cj = j * sy + kv * V;
    // Odd chunks walk their planes downwards: a boundary plane between two
    // chunks is then read by both at the same step (both ends of the walks
    // meet there), so the second read can come from the L2.  Walking
    // direction changes which registers hold the x neighbours, never the
    // arithmetic of a cell.
    const int dir = (ch & 1u) ? -1 : 1;
    const int s0 = dir > 0 ? ((int)i0 > 0 ? (int)i0 - 1 : 0) : ((int)i1 < (int)nx ? (int)i1 : (int)nx - 1);
    const int se = dir > 0 ? (int)i1 : (int)i0 - 1;
    // q of planes s-2d, s-d, s; x0 of s-d, s; colour-A results of s-2d, s-d;
    // r, 1/diag and the y-neighbour term of s-d (d = dir)
    T qa[V], qb[V], qc[V], xb[V], xc[V], ma[V], mb[V], rb[V], ib[V], yb[V];
    {
      const unsigned fb = (unsigned)clampp(s0 - dir) * P + cj, fc = (unsigned)s0 * P + cj;
      if (CQ) {
        fillq(qb);
        fillq(qc);
      } else {
        ldv<T>(at(L.qc, fb), qb);
        ldv<T>(at(L.qc, fc), qc);
      }
      if (X0) {
        lx(fb, xb);
        lx(fc, xc);
      } else {
        zero(xb);
        zero(xc);
      }
      copy(qa, qb);
      zero(ma);
      zero(mb);
      zero(rb);
      zero(yb);
#pragma unroll
      for (int v = 0; v < V; ++v) ib[v] = 1;
    }
    T pqzm = 0, pqzp = 0;   // WE: z neighbours' q of plane s - dir
    for (int s = s0;; s += dir) {
      const bool live = s >= 0 && s < (int)nx;   // s = nx or -1 only finishes the chunk's last plane
      const unsigned c = (unsigned)clampp(s) * P + cj;
      const bool hxm = s > 0, hxp = s + 1 < (int)nx;
      const unsigned fn = (unsigned)clampp(s + dir) * P + cj, fym = hym ? c - sy : c, fyp = hyp ? c + sy : c;
      T qd[V], xd[V], rc[V], nqm[V], nqp[V], nxm[V], nxp[V];
      if (CQ) fillq(qd);
      else ldv<T>(at(L.qc, fn), qd);
      if (X0) lx(fn, xd);
      else zero(xd);
      ldv<T>(at(r, c), rc);
      if (!inm) {
        if (!CQ) ldv<T>(at(L.qc, fym), nqm);
        if (X0) lx(fym, nxm);
      }
      if (!inp) {
        if (!CQ) ldv<T>(at(L.qc, fyp), nqp);
        if (X0) lx(fyp, nxp);
      }
      if (!CQ) stv<T>(&lsq[par][tid * V], qc);
      if (X0) stv<T>(&lsx[par][tid * V], xc);
      if (WE) {
        lsm[par][2 * tid] = mb[0];
        lsm[par][2 * tid + 1] = mb[V - 1];
      }
      __syncthreads();
      if (inm) {
        if (!CQ) ldv<T>(&lsq[par][(tid - (int)nzv) * V], nqm);
        if (X0) ldv<T>(&lsx[par][(tid - (int)nzv) * V], nxm);
      }
      if (inp) {
        if (!CQ) ldv<T>(&lsq[par][(tid + (int)nzv) * V], nqp);
        if (X0) ldv<T>(&lsx[par][(tid + (int)nzv) * V], nxp);
      }
      if (CQ) {
        fillq(nqm);
        fillq(nqp);
      }
      if (!X0) {
        zero(nxm);
        zero(nxp);
      }
      // z neighbours from the adjacent lanes; at a wave's first and last lane
      // (rows longer than or straddling a wave) from the adjacent thread's
      // values in LDS
      T qzm = CQ ? qk : lane_up(qc[V - 1]), qzp = CQ ? qk : lane_down(qc[0]);
      T xzm = lane_up(xc[V - 1]), xzp = lane_down(xc[0]);
      T mzm = lane_up(mb[V - 1]), mzp = lane_down(mb[0]);
      if (WE && hzm && lane == 0) {
        if (!CQ) qzm = lsq[par][(tid - 1) * V + V - 1];
        if (X0) xzm = lsx[par][(tid - 1) * V + V - 1];
        mzm = lsm[par][2 * (tid - 1) + 1];
      }
      if (WE && hzp && lane == 63) {
        if (!CQ) qzp = lsq[par][(tid + 1) * V];
        if (X0) xzp = lsx[par][(tid + 1) * V];
        mzp = lsm[par][2 * (tid + 1)];
      }
      par ^= 1;
      // x neighbours of plane s: minus side, plus side
      const bool fw = dir > 0;
      // the y-neighbour term and 1/diag of plane s (diag formed in T from q:
      // the smoother's own diagonal, consistent within the sweep)
      T yc[V], ic[V];
#pragma unroll
      for (int v = 0; v < V; ++v) {
        T ty = 0;
        ty = hym ? ty + (qc[v] + nqm[v]) * nxm[v] : ty;
        ty = hyp ? ty + (qc[v] + nqp[v]) * nxp[v] : ty;
        yc[v] = ty;
      }
      if (L.dfly) {
        const int dm = L.dmask;
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const T q = qc[v], bnd = T(2) * L.sc * q;
          const T gxm = fw ? qb[v] : qd[v], gxp = fw ? qd[v] : qb[v];
          T d = 0;
          d += hxm ? hs * (q + gxm) : ((dm & 1) ? bnd : T(0));
          d += hxp ? hs * (q + gxp) : ((dm & 2) ? bnd : T(0));
          d += hym ? hs * (q + nqm[v]) : ((dm & 4) ? bnd : T(0));
          d += hyp ? hs * (q + nqp[v]) : ((dm & 8) ? bnd : T(0));
          const bool em = v > 0 || hzm, ep = v < V - 1 || hzp;
          const T gm = v > 0 ? qc[v > 0 ? v - 1 : 0] : qzm;
          const T gp = v < V - 1 ? qc[v < V - 1 ? v + 1 : V - 1] : qzp;
          d += em ? hs * (q + gm) : ((dm & 16) ? bnd : T(0));
          d += ep ? hs * (q + gp) : ((dm & 32) ? bnd : T(0));
          ic[v] = T(1) / d;
        }
      } else {
        T dl[V];
        ldv<T>(at(L.diag, c), dl);
#pragma unroll
        for (int v = 0; v < V; ++v) ic[v] = T(1) / dl[v];
      }
      const T bqzm = CQ ? qk : (WE ? pqzm : lane_up(qb[V - 1])), bqzp = CQ ? qk : (WE ? pqzp : lane_down(qb[0]));
      const T w1 = T(1) - w;
      T mc[V];
      const int sb = s - dir;   // the plane colour B finishes
      const bool own_b = sb >= (int)i0 && sb < (int)i1;
      // x + w (r - A x)/d = (1 - w) x + w (r + sc/2 off)/d, off the neighbour
      // sum.  The lanes of colour A on plane s are those of colour B on plane
      // s - dir (v of parity s + c0); each lane evaluates only its colour.
      auto relax = [&](auto PA) {
        constexpr unsigned pa = decltype(PA)::value;
        // colour A on plane s, from x0 (all neighbours old)
#pragma unroll
        for (int v = 0; v < V; ++v) {
          if (((unsigned)v & 1u) == pa) {
            const T gxm = fw ? qb[v] : qd[v], gxp = fw ? qd[v] : qb[v];
            const T vxm = fw ? xb[v] : xd[v], vxp = fw ? xd[v] : xb[v];
            T o = yc[v];
            o = hxm ? o + (qc[v] + gxm) * vxm : o;
            o = hxp ? o + (qc[v] + gxp) * vxp : o;
            const T gm = v > 0 ? qc[v > 0 ? v - 1 : 0] : qzm, xm = v > 0 ? xc[v > 0 ? v - 1 : 0] : xzm;
            const T gp = v < V - 1 ? qc[v < V - 1 ? v + 1 : V - 1] : qzp;
            const T xp = v < V - 1 ? xc[v < V - 1 ? v + 1 : V - 1] : xzp;
            o = (v > 0 || hzm) ? o + (qc[v] + gm) * xm : o;
            o = (v < V - 1 || hzp) ? o + (qc[v] + gp) * xp : o;
            mc[v] = w1 * xc[v] + w * ic[v] * (rc[v] + hs * o);
          } else {
            mc[v] = xc[v];
          }
        }
        // colour B on plane s - dir, from colour A's new values (y old)
        if (own_b) {
          const bool bxm = sb > 0, bxp = sb + 1 < (int)nx;
          T o[V];
#pragma unroll
          for (int v = 0; v < V; ++v) {
            if (((unsigned)v & 1u) == pa) {
              const T gxm = fw ? qa[v] : qc[v], gxp = fw ? qc[v] : qa[v];
              const T vxm = fw ? ma[v] : mc[v], vxp = fw ? mc[v] : ma[v];
              T f = yb[v];
              f = bxm ? f + (qb[v] + gxm) * vxm : f;
              f = bxp ? f + (qb[v] + gxp) * vxp : f;
              const T gm = v > 0 ? qb[v > 0 ? v - 1 : 0] : bqzm, xm = v > 0 ? mb[v > 0 ? v - 1 : 0] : mzm;
              const T gp = v < V - 1 ? qb[v < V - 1 ? v + 1 : V - 1] : bqzp;
              const T xp = v < V - 1 ? mb[v < V - 1 ? v + 1 : V - 1] : mzp;
              f = (v > 0 || hzm) ? f + (qb[v] + gm) * xm : f;
              f = (v < V - 1 || hzp) ? f + (qb[v] + gp) * xp : f;
              o[v] = w1 * mb[v] + w * ib[v] * (rb[v] + hs * f);
            } else {
              o[v] = mb[v];
            }
          }
          out((unsigned)sb * P + cj, o, rb);
        }
      };
      if ((((unsigned)s + (unsigned)c0) & 1u) == 0u) relax(std::integral_constant<unsigned, 0>{});
      else relax(std::integral_constant<unsigned, 1>{});
      (void)live;
      copy(qa, qb);
      copy(qb, qc);
      copy(qc, qd);
      copy(xb, xc);
      copy(xc, xd);
      copy(ma, mb);
      copy(mb, mc);
      copy(rb, rc);
      copy(ib, ic);
      copy(yb, yc);
      if (WE) {
        pqzm = qzm;
        pqzp = qzp;
      }
      if (s == se) break;
    }
  }
}

// Levels that take the coloured sweeps: rows shared through LDS (each z-row
// inside one block) and chunks of at least min_planes x-planes (a chunk also
// relaxes colour A on its two outer planes, which short chunks pay for more
// than the better smoothing saves: at 128^3 the chunks are 2 planes long).
template <class T>
inline bool rb_marching_ok(const Lev<T>& M, int min_planes) {   // M: the level as march_lev(L, 1) returns it
  // FP32 levels only: in FP64 the kernel holds twice the registers per
  // vector and spills (FP64 fine level at 256^3: 35.4 -> 36.6 ms per step)
  if (!std::is_same<T, float>::value || !use_vec(M)) return false;
  const long long nzv = M.nz / VW<T>::n;
  const long long clen = (M.nx + M.mch - 1) / M.mch;
  return nzv >= 1 && M.mnt % nzv == 0 && ((long long)M.ny * nzv) % M.mnt == 0 && clen >= min_planes;
}

enum { RB_GEN = 0, RB_ZERO = 1, RB_PROLONG = 2 };

// Do the level's z-rows span or straddle 64-lane waves (the coloured sweep
// then exchanges wave-edge values through LDS)?
template <class T>
inline bool rows_cross_waves(const Lev<T>& M) {
  const int nzv = M.nz / VW<T>::n;
  return 64 % nzv != 0;
}

// One coloured sweep (march_rb) of F x = r.  RB_GEN: from x; RB_ZERO: from
// x = 0 (x not read); RB_PROLONG: from x + P xc (injection from level C).
// DOT: also <r, x_out> (the preconditioned residual's product).
template <class T, int MODE, bool DOT, int NT, bool WE, bool CQ = false>
VEC_KERNEL_M k_mg_rb_v(Lev<T> F, Lev<T> C, const T* __restrict__ r, const T* __restrict__ x,
                       const T* __restrict__ xc, T* __restrict__ xout, T w, int c0, SolveStatus* st,
                       double* partials, unsigned* counter, int first) {
  if (st->done) return;
  constexpr int V = VW<T>::n;
  double acc = 0.0;
  auto outf = [&](unsigned c, const T(&o)[V], const T(&rv)[V]) {
    stv<T>(at(xout, c), o);
    if (DOT) {
#pragma unroll
      for (int v = 0; v < V; ++v) acc += (double)rv[v] * (double)o[v];
    }
  };
  if constexpr (MODE == RB_PROLONG) {
    auto row = [&](unsigned f, T(&o)[V]) {
      const unsigned rr = f / (unsigned)F.nz;   // ii*ny + jj
      const unsigned kk = f - rr * (unsigned)F.nz;
      const unsigned jj = rr % (unsigned)F.ny, ii = rr / (unsigned)F.ny;
      const unsigned pb = ((ii >> 1) * (unsigned)C.ny + (jj >> 1)) * (unsigned)C.nz + (kk >> 1);
      ldv<T>(at(x, f), o);
#pragma unroll
      for (int v = 0; v < V; ++v) o[v] += *at(xc, pb + (v >> 1));
    };
    march_rb<T, NT, true, WE, CQ>(F, r, w, c0, row, outf);
  } else if constexpr (MODE == RB_GEN) {
    march_rb<T, NT, true, WE, CQ>(F, r, w, c0, [&](unsigned f, T(&o)[V]) { ldv<T>(at(x, f), o); }, outf);
  } else {
    march_rb<T, NT, false, WE, CQ>(F, r, w, c0, [&](unsigned, T(&o)[V]) {}, outf);
  }
  if (DOT) publish_rz<NT>(acc, st, partials, counter, first);
}

// r32 (may be null): also r in FP32 (the V-cycle's input at the start of a
// solve in the FP32-multigrid form).
// CQ: the coefficient is L.qk in every cell (no q loads).  r may be null
// (the status only).
template <int NT, bool CQ = false>
VEC_KERNEL_M k_resid64_v(Lev<double> L, const double* __restrict__ b, const double* __restrict__ x,
                       double* __restrict__ r, SolveStatus* st, double* partials, unsigned* counter, int set_bnorm,
                       float* __restrict__ r32) {
  constexpr int V = VW<double>::n;
  double acc[2] = {0.0, 0.0};
  march<double, NT, true, CQ>(
      L, [&](unsigned f, double(&o)[V]) { ldv<double>(at(x, f), o); }, [&](unsigned f) { return *at(x, f); },
      [&](unsigned c, const double(&qv)[V], const double(&xv)[V], const double(&off)[V], const double(&dg)[V]) {
        double bv[V], o[V];
        ldv<double>(at(b, c), bv);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          const double ax = dg[v] * xv[v] - 0.5 * L.sc * off[v];
          o[v] = bv[v] - ax;
          acc[0] += bv[v] * bv[v];
          acc[1] += o[v] * o[v];
        }
        if (r) stv<double>(at(r, c), o);
        if (r32) {
          float2 rf;
          rf.x = (float)o[0];
          rf.y = (float)o[1];
          *reinterpret_cast<float2*>(at(r32, c)) = rf;
        }
      });
  const int ops[2] = {RSUM, RSUM};
  if (block_reduce_publish<2, NT>(acc, ops, partials, counter)) {
    double t[2];
    block_combine<2, NT>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      if (set_bnorm) {
        st->bb = t[0];
        st->bnorm = sqrt(t[0]);
        st->it = 0;
      }
      st->rr = t[1];
      st->zero = st->bb == 0.0;
      st->res = st->bb == 0.0 ? 0.0 : sqrt(t[1]) / st->bnorm;
      st->done = (st->bb == 0.0 || st->res <= st->tol) ? 1 : 0;
    }
  }
}

template <class T>
VEC_KERNEL k_inner_init_v(Lev<T> L, const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ x,
                               SolveStatus* st, double* partials, unsigned* counter) {
  constexpr int V = VW<T>::n;
  double acc[1] = {0.0};
  FOR_ITEMS(L, T, i, j, kv, c) {
    T rv[V], zv[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      rv[v] = (T)*at(r64, c + v);
      zv[v] = 0;
      acc[0] += (double)rv[v] * (double)rv[v];
    }
    stv<T>(at(r, c), rv);
    stv<T>(at(x, c), zv);
  }
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double t[1];
    block_combine<1>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      st->bb = t[0];
      st->bnorm = sqrt(t[0]);
      st->rr = t[0];
      st->res = t[0] == 0.0 ? 0.0 : 1.0;
      st->it = 0;
      st->zero = t[0] == 0.0;
      st->done = t[0] == 0.0 ? 1 : 0;
    }
  }
}

// k_inner_init_v and k_jac_rz_v in one pass (a Jacobi-preconditioned round
// of the precision form): r = (T) r64, x = 0, z = r/diag; ||r||^2 and <r, z>.
template <class T>
VEC_KERNEL k_inner_init_jac_v(Lev<T> L, const double* __restrict__ r64, T* __restrict__ r, T* __restrict__ x,
                              T* __restrict__ zout, SolveStatus* st, double* partials, unsigned* counter) {
  constexpr int V = VW<T>::n;
  double acc[2] = {0.0, 0.0};
  FOR_ITEMS(L, T, i, j, kv, c) {
    T rv[V], xv[V], dv[V], zv[V];
    ldv<T>(at(L.diag, c), dv);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      rv[v] = (T)*at(r64, c + v);
      xv[v] = 0;
      acc[0] += (double)rv[v] * (double)rv[v];
      acc[1] += (double)rv[v] * (double)rv[v] / (double)dv[v];
      zv[v] = rv[v] / dv[v];
    }
    stv<T>(at(r, c), rv);
    stv<T>(at(x, c), xv);
    if (zout) stv<T>(at(zout, c), zv);
  }
  const int ops[2] = {RSUM, RSUM};
  if (block_reduce_publish<2>(acc, ops, partials, counter)) {
    double t[2];
    block_combine<2>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      st->bb = t[0];
      st->bnorm = sqrt(t[0]);
      st->rr = t[0];
      st->res = t[0] == 0.0 ? 0.0 : 1.0;
      st->it = 0;
      st->zero = t[0] == 0.0;
      st->done = t[0] == 0.0 ? 1 : 0;
      st->rz = t[1];
    }
  }
}

template <class T>
VEC_KERNEL k_jac_rz_v(Lev<T> L, const T* __restrict__ r, SolveStatus* st, double* partials, unsigned* counter,
                           int first, T* __restrict__ zout) {
  if (st->done) return;
  constexpr int V = VW<T>::n;
  double acc = 0.0;
  FOR_ITEMS(L, T, i, j, kv, c) {
    T rv[V], dv[V], zv[V];
    ldv<T>(at(r, c), rv);
    ldv<T>(at(L.diag, c), dv);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      acc += (double)rv[v] * (double)rv[v] / (double)dv[v];
      zv[v] = rv[v] / dv[v];
    }
    if (zout) stv<T>(at(zout, c), zv);
  }
  publish_rz(acc, st, partials, counter, first);
}

// FIRST: p = z (the first iteration).  x (may be null): also x += alpha_prev
// p_old, the previous iteration's deferred solution update (alpha_prev is
// still in st->alpha when this kernel starts; its last block replaces it).
template <class T, bool JAC, bool FIRST, int NT>
VEC_KERNEL_M k_cg_dir_spmv_v(Lev<T> L, const T* __restrict__ z, const T* __restrict__ r,
                           const T* __restrict__ pin, T* __restrict__ pout, T* __restrict__ q, SolveStatus* st,
                           double* partials, unsigned* counter, T* __restrict__ x) {
  if (st->done) return;
  constexpr int V = VW<T>::n;
  const T be = FIRST ? T(0) : (T)st->beta;
  const T ap = FIRST ? T(0) : (T)st->alpha;
  double acc[1] = {0.0};
  auto pnv = [&](unsigned f, T(&o)[V]) {
    if (JAC) {
      T rv[V], dv[V];
      ldv<T>(at(r, f), rv);
      ldv<T>(at(L.diag, f), dv);
#pragma unroll
      for (int v = 0; v < V; ++v) o[v] = rv[v] / dv[v];
    } else {
      ldv<T>(at(z, f), o);
    }
    if (!FIRST) {
      T pv[V];
      ldv<T>(at(pin, f), pv);
#pragma unroll
      for (int v = 0; v < V; ++v) o[v] = o[v] + be * pv[v];
    }
  };
  auto pns = [&](unsigned f) -> T {
    const T zf = JAC ? *at(r, f) / *at(L.diag, f) : *at(z, f);
    return FIRST ? zf : zf + be * *at(pin, f);
  };
  march<T, NT>(L, pnv, pns, [&](unsigned c, const T(&qv)[V], const T(&pc)[V], const T(&off)[V], const T(&dv)[V]) {
    T y[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      y[v] = dv[v] * pc[v] - T(0.5) * L.sc * off[v];
      acc[0] += (double)pc[v] * (double)y[v];
    }
    stv<T>(at(pout, c), pc);
    stv<T>(at(q, c), y);
    if (!FIRST && x) {
      T xv[V], pv[V];
      ldv<T>(at(x, c), xv);
      ldv<T>(at(pin, c), pv);
#pragma unroll
      for (int v = 0; v < V; ++v) xv[v] += ap * pv[v];
      stv<T>(at(x, c), xv);
    }
  });
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1, NT>(acc, ops, partials, counter)) {
    double t[1];
    block_combine<1, NT>(ops, partials, counter, t);
    if (threadIdx.x == 0) st->alpha = st->rz / t[0];
  }
}

template <class T, bool JAC, int NT>
static auto dir_v(bool first) {
  return first ? k_cg_dir_spmv_v<T, JAC, true, NT> : k_cg_dir_spmv_v<T, JAC, false, NT>;
}

// Calls f(std::integral_constant<int, NT>) for the level's marching block size.
template <class F>
inline void with_nt(int nt, F&& f) {
  if (nt == 512) f(std::integral_constant<int, 512>{});
  else if (nt == 384) f(std::integral_constant<int, 384>{});
  else f(std::integral_constant<int, 256>{});
}

template <class T, bool JAC>
VEC_KERNEL k_cg_update_v(Lev<T> L, T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p,
                              const T* __restrict__ q, SolveStatus* st, double* partials, unsigned* counter,
                              T* __restrict__ zout) {
  if (st->done) return;
  constexpr int V = VW<T>::n;
  const T a = (T)st->alpha;
  double acc[2] = {0.0, 0.0};
  // x null: the solution update is deferred to the next direction update
  FOR_ITEMS(L, T, i, j, kv, c) {
    T xv[V], rv[V], pv[V], qv[V];
    if (x) {
      ldv<T>(at(x, c), xv);
      ldv<T>(at(p, c), pv);
    }
    ldv<T>(at(r, c), rv);
    ldv<T>(at(q, c), qv);
    T dv[V], zv[V];
    if (JAC) ldv<T>(at(L.diag, c), dv);
#pragma unroll
    for (int v = 0; v < V; ++v) {
      if (x) xv[v] += a * pv[v];
      rv[v] = rv[v] - a * qv[v];
      acc[0] += (double)rv[v] * (double)rv[v];
      if (JAC) {
        acc[1] += (double)rv[v] * (double)rv[v] / (double)dv[v];
        zv[v] = rv[v] / dv[v];
      }
    }
    if (x) stv<T>(at(x, c), xv);
    stv<T>(at(r, c), rv);
    if (JAC && zout) stv<T>(at(zout, c), zv);
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
      } else if (JAC) {
        st->beta = t[1] / st->rz;
        st->rz = t[1];
      }
    }
  }
}

// Residual update with the first-order Neumann-series polynomial preconditioner
// of the Jacobi splitting A = D - N:
//   r' = r - alpha q,   y = D^-1 r',   z = D^-1 (r' + N y)  (= (D^-1 + D^-1 N D^-1) r'),
// with N y = sc/2 sum_nb (q_c + q_nb) y_nb formed by the marching stencil
// from the neighbours' r - alpha q and diag.  For the diagonally dominant
// energy and species systems the spectrum of D^-1 A lies in [1 - b, 1 + b]
// with b < 1, and that of M^-1 A = I - (D^-1 N)^2 in [1 - b^2, 1], which
// roughly halves the CG iterations for one stencil pass more in this kernel.
// Neighbours read r, so r' goes to a second buffer (rout).  INIT: alpha = 0
// and no q (the first z of a solve); rout is not written and only rz is set.
// Also <r', r'> (convergence test) and <r', z> (beta), as k_cg_update_v.
template <class T, bool INIT, int NT>
VEC_KERNEL_M k_cg_update_neu_v(Lev<T> L, const T* __restrict__ rin, T* __restrict__ rout, const T* __restrict__ q,
                               T* __restrict__ zout, SolveStatus* st, double* partials, unsigned* counter) {
  if (st->done) return;
  constexpr int V = VW<T>::n;
  const T a = INIT ? T(0) : (T)st->alpha;
  double acc[2] = {0.0, 0.0};
  auto rn_at = [&](unsigned f, T(&o)[V]) {
    ldv<T>(at(rin, f), o);
    if (!INIT) {
      T qv[V];
      ldv<T>(at(q, f), qv);
#pragma unroll
      for (int v = 0; v < V; ++v) o[v] = o[v] - a * qv[v];
    }
  };
  march<T, NT>(
      L,
      [&](unsigned f, T(&o)[V]) {
        T dv[V];
        rn_at(f, o);
        ldv<T>(at(L.diag, f), dv);
#pragma unroll
        for (int v = 0; v < V; ++v) o[v] = o[v] / dv[v];
      },
      [&](unsigned f) -> T { return (INIT ? *at(rin, f) : *at(rin, f) - a * *at(q, f)) / *at(L.diag, f); },
      [&](unsigned c, const T(&qv)[V], const T(&yv)[V], const T(&off)[V], const T(&dv)[V]) {
        T rv[V], zv[V];
        rn_at(c, rv);
#pragma unroll
        for (int v = 0; v < V; ++v) {
          zv[v] = (rv[v] + T(0.5) * L.sc * off[v]) / dv[v];
          acc[0] += (double)rv[v] * (double)rv[v];
          acc[1] += (double)rv[v] * (double)zv[v];
        }
        if (!INIT) stv<T>(at(rout, c), rv);
        stv<T>(at(zout, c), zv);
      });
  const int ops[2] = {RSUM, RSUM};
  if (block_reduce_publish<2, NT>(acc, ops, partials, counter)) {
    double t[2];
    block_combine<2, NT>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      if (INIT) {
        st->rz = t[1];
      } else {
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
}

// FP64 CG with the FP32 multigrid preconditioner: the update also stores
// r in FP32 for the V-cycle; the direction update reads z in FP32.  The
// solution update x += alpha p is deferred to the next direction update,
// which reads p anyway (and, after the last iteration, to k_axpy_alpha), so
// this kernel streams r and q only.
VEC_KERNEL k_cg_update_r32_v(Lev<double> L, double* __restrict__ r, const double* __restrict__ q,
                             float* __restrict__ r32, SolveStatus* st, double* partials, unsigned* counter) {
  if (st->done) return;
  constexpr int V = VW<double>::n;
  const double a = st->alpha;
  double acc[1] = {0.0};
  FOR_ITEMS(L, double, i, j, kv, c) {
    double rv[V], qv[V];
    ldv<double>(at(r, c), rv);
    ldv<double>(at(q, c), qv);
    float2 rf;
#pragma unroll
    for (int v = 0; v < V; ++v) {
      rv[v] = rv[v] - a * qv[v];
      acc[0] += rv[v] * rv[v];
    }
    rf.x = (float)rv[0];
    rf.y = (float)rv[1];
    stv<double>(at(r, c), rv);
    *reinterpret_cast<float2*>(at(r32, c)) = rf;
  }
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1>(acc, ops, partials, counter)) {
    double t[1];
    block_combine<1>(ops, partials, counter, t);
    if (threadIdx.x == 0) {
      st->it += 1;
      st->rr = t[0];
      st->res = sqrt(t[0]) / st->bnorm;
      if (st->res <= st->tol) st->done = 1;
      else if (st->it >= st->maxit) st->done = 2;
    }
  }
}

// x (may be null): also x += alpha_prev p_old, the previous iteration's
// solution update (alpha_prev is still in st->alpha when this kernel starts;
// its last block replaces it).
template <bool FIRST, int NT, bool CQ = false>
VEC_KERNEL_M k_cg_dir_spmv_z32_v(Lev<double> L, const float* __restrict__ z, const float* __restrict__ pin,
                               float* __restrict__ pout, double* __restrict__ q, SolveStatus* st,
                               double* partials, unsigned* counter, double* __restrict__ x) {
  if (st->done) return;
  constexpr int V = VW<double>::n;
  const double be = FIRST ? 0.0 : st->beta;
  const double ap = FIRST ? 0.0 : st->alpha;
  double acc[1] = {0.0};
  // p = z + beta p_old formed in FP64 and stored in FP32; the operator, q and
  // the dot products use that FP32 value exactly (every thread rounds alike)
  auto pnv = [&](unsigned f, double(&o)[V]) {
    const float2 zf = *reinterpret_cast<const float2*>(at(z, f));
    if (FIRST) {
      o[0] = (double)zf.x;
      o[1] = (double)zf.y;
    } else {
      const float2 pf = *reinterpret_cast<const float2*>(at(pin, f));
      o[0] = (double)(float)((double)zf.x + be * (double)pf.x);
      o[1] = (double)(float)((double)zf.y + be * (double)pf.y);
    }
  };
  auto pns = [&](unsigned f) -> double {
    return FIRST ? (double)*at(z, f) : (double)(float)((double)*at(z, f) + be * (double)*at(pin, f));
  };
  march<double, NT, true, CQ>(L, pnv, pns,
                [&](unsigned c, const double(&qv)[V], const double(&pc)[V], const double(&off)[V],
                    const double(&dv)[V]) {
    double y[V];
#pragma unroll
    for (int v = 0; v < V; ++v) {
      y[v] = dv[v] * pc[v] - 0.5 * L.sc * off[v];
      acc[0] += pc[v] * y[v];
    }
    *reinterpret_cast<float2*>(at(pout, c)) = make_float2((float)pc[0], (float)pc[1]);
    stv<double>(at(q, c), y);
    if (!FIRST && x) {
      double xv[V];
      ldv<double>(at(x, c), xv);
      const float2 pf = *reinterpret_cast<const float2*>(at(pin, c));
      xv[0] += ap * (double)pf.x;
      xv[1] += ap * (double)pf.y;
      stv<double>(at(x, c), xv);
    }
  });
  const int ops[1] = {RSUM};
  if (block_reduce_publish<1, NT>(acc, ops, partials, counter)) {
    double t[1];
    block_combine<1, NT>(ops, partials, counter, t);
    if (threadIdx.x == 0) st->alpha = st->rz / t[0];
  }
}

// x += st->alpha p: the last iteration's deferred solution update (runs
// after the solve has been flagged done).
template <class T>
__global__ void k_axpy_alpha(T* __restrict__ x, const T* __restrict__ p, const SolveStatus* st, long long n) {
  const T a = (T)st->alpha;
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) x[e] += a * p[e];
}
template <class T>
void launch_axpy_alpha(T* x, const T* p, const SolveStatus* st, long long n, hipStream_t s) {
  k_axpy_alpha<T><<<grid_blocks(n), BLOCK, 0, s>>>(x, p, st, n);
}
template void launch_axpy_alpha<double>(double*, const double*, const SolveStatus*, long long, hipStream_t);
template void launch_axpy_alpha<float>(float*, const float*, const SolveStatus*, long long, hipStream_t);
__global__ void k_axpy_alpha_p32(double* __restrict__ x, const float* __restrict__ p, const SolveStatus* st,
                                 long long n) {
  const double a = st->alpha;
  long long b0, b1;
  block_range(n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) x[e] += a * (double)p[e];
}
void launch_axpy_alpha(double* x, const float* p, const SolveStatus* st, long long n, hipStream_t s) {
  k_axpy_alpha_p32<<<grid_blocks(n), BLOCK, 0, s>>>(x, p, st, n);
}

// x += e; with p, first e += alpha p (the inner solve's last deferred update,
// alpha from st), as launch_axpy_alpha followed by the plain correction.
template <class T>
VEC_KERNEL k_add_correction_v(Lev<T> L, double* __restrict__ x, const T* __restrict__ e, const T* __restrict__ p,
                              const SolveStatus* st, const T* __restrict__ p_odd) {
  constexpr int V = VW<T>::n;
  // p_odd set: the deferred direction is p_odd or p (even) by the parity of
  // the device's iteration count, none before the first iteration
  if (p_odd) p = st->it > 0 ? ((st->it & 1) ? p_odd : p) : nullptr;
  const T a = p ? (T)st->alpha : T(0);
  FOR_ITEMS(L, T, i, j, kv, c) {
    T ev[V], pv[V];
    ldv<T>(at(e, c), ev);
    if (p) {
      ldv<T>(at(p, c), pv);
#pragma unroll
      for (int v = 0; v < V; ++v) ev[v] += a * pv[v];
    }
#pragma unroll
    for (int v = 0; v < V; ++v) *at(x, c + v) += (double)ev[v];
  }
}

// ------------------------------------------------------------ host side
template <class T>
void mg_setup_levels(MgHier<T>& H, int dirmask, hipStream_t s) {
  for (int l = 0; l < H.nlev; ++l) {
    H.lev[l].dfly = 1;
    H.lev[l].dmask = dirmask;
  }
  for (int l = 1; l < H.nlev; ++l) {
    Lev<T>& C = H.lev[l];
    k_mg_coarsen_q<T><<<tile_blocks(C.ntiles), BLOCK, 0, s>>>(H.lev[l - 1], C, const_cast<T*>(C.qc));
    k_mg_diag<T><<<tile_blocks(C.ntiles), BLOCK, 0, s>>>(C, dirmask, const_cast<T*>(C.diag));
  }
}

// ------------------------------------------------------- V-cycle tail in LDS
// The coarse end of the V-cycle -- every level from some level down, when
// their r, x, t, q, diag all fit in one workgroup's LDS -- runs as one launch
// of one 1024-thread workgroup: the same sweeps, restriction and injection as
// the per-level kernels, each pass followed by a workgroup barrier.  It
// replaces about nine launches of a few microseconds per V-cycle.
constexpr int TAIL_BLOCK = 1024;
constexpr size_t TAIL_LDS_MAX = 96 * 1024;

template <class T>
struct TailLevs {
  int nlev;
  int nx[MG_MAXLEV], ny[MG_MAXLEV], nz[MG_MAXLEV], nu[MG_MAXLEV];
  int ly[MG_MAXLEV], lz[MG_MAXLEV];   // log2 of ny, nz when both are powers of two, else -1
  int off[MG_MAXLEV];   // element offset of the level's r, x, t, q, 1/diag block in LDS
  T sc[MG_MAXLEV];
  const T* q[MG_MAXLEV];
  const T* d[MG_MAXLEV];
};

template <class T>
inline size_t tail_bytes(const MgHier<T>& H, int l) {
  size_t b = 0;
  for (int m = l; m < H.nlev; ++m) b += 5 * (size_t)H.lev[m].n * sizeof(T);
  return b;
}

// DOT: the last sweep on the first tail level publishes <r, x> (the tail
// then starts at the hierarchy's finest level).  Arrays are addressed by
// offsets into the LDS block (no pointer tables); bit l of `flip` says that
// level l's iterate currently sits in its t array.
template <class T, bool DOT>
__global__ void __launch_bounds__(TAIL_BLOCK) k_mg_tail(TailLevs<T> TL, const T* __restrict__ r0,
                                                        T* __restrict__ xout, T omega, int coarse_sweeps,
                                                        SolveStatus* st, int first) {
  if (st->done) return;
  extern __shared__ double tail_smem[];
  T* S = reinterpret_cast<T*>(tail_smem);
  const int L = TL.nlev;
  unsigned flip = 0;
  auto N = [&](int l) { return TL.nx[l] * TL.ny[l] * TL.nz[l]; };
  auto Ro = [&](int l) { return TL.off[l]; };
  auto Xo = [&](int l) { return TL.off[l] + N(l) * (1 + (int)((flip >> l) & 1u)); };
  auto Yo = [&](int l) { return TL.off[l] + N(l) * (2 - (int)((flip >> l) & 1u)); };
  auto Qo = [&](int l) { return TL.off[l] + 3 * N(l); };
  auto Do = [&](int l) { return TL.off[l] + 4 * N(l); };
  for (int l = 0; l < L; ++l) {
    const int n = N(l), qo = Qo(l), dg = Do(l);
    for (int c = threadIdx.x; c < n; c += TAIL_BLOCK) {
      S[qo + c] = TL.q[l][c];
      S[dg + c] = T(1) / TL.d[l][c];   // 1/diag: the sweeps multiply
    }
  }
  for (int c = threadIdx.x; c < N(0); c += TAIL_BLOCK) S[Ro(0) + c] = r0[c];
  __syncthreads();
  double acc = 0.0;
  // c -> (i, j, k) on an a x b x m level without integer division: with the
  // offset of one half, (c + 1/2)/m lies at least 1/(2m) from an integer, far
  // beyond the FP64 rounding of the product (c < 2^24 here).
  auto dec = [](int c, int b, int m, int& i, int& j, int& k) {
    const int t = (int)(((double)c + 0.5) * (1.0 / (double)m));
    k = c - t * m;
    i = (int)(((double)t + 0.5) * (1.0 / (double)b));
    j = t - i * b;
  };
  // the same by shifts on levels with power-of-two ny, nz
  auto decl = [&](int l, int c, int& i, int& j, int& k) {
    if (TL.lz[l] >= 0) {
      k = c & (TL.nz[l] - 1);
      const int t = c >> TL.lz[l];
      j = t & (TL.ny[l] - 1);
      i = t >> TL.ly[l];
    } else {
      dec(c, TL.ny[l], TL.nz[l], i, j, k);
    }
  };
  // one damped-Jacobi sweep on level l (x -> t, then the roles swap); with
  // dot, accumulate <r, x_new>.  zero: from x = 0, i.e. x = omega r/diag.
  // x + omega (r - A x)/d is formed as (1 - omega) x + omega (r + sc/2 off)/d.
  auto sweep = [&](int l, bool zero, bool dot) {
    const int nx = TL.nx[l], ny = TL.ny[l], nz = TL.nz[l], n = nx * ny * nz, sx = ny * nz;
    const int ro = Ro(l), xo = Xo(l), yo = Yo(l), qo = Qo(l), dg = Do(l);
    const T sc = TL.sc[l];
    for (int c = threadIdx.x; c < n; c += TAIL_BLOCK) {
      T xn;
      if (zero) {
        xn = omega * S[ro + c] * S[dg + c];
      } else {
        int i, j, k;
        decl(l, c, i, j, k);
        const T q = S[qo + c];
        T off = 0;
        if (i > 0) off += (q + S[qo + c - sx]) * S[xo + c - sx];
        if (i < nx - 1) off += (q + S[qo + c + sx]) * S[xo + c + sx];
        if (j > 0) off += (q + S[qo + c - nz]) * S[xo + c - nz];
        if (j < ny - 1) off += (q + S[qo + c + nz]) * S[xo + c + nz];
        if (k > 0) off += (q + S[qo + c - 1]) * S[xo + c - 1];
        if (k < nz - 1) off += (q + S[qo + c + 1]) * S[xo + c + 1];
        xn = (T(1) - omega) * S[xo + c] + omega * (S[ro + c] + T(0.5) * sc * off) * S[dg + c];
      }
      S[yo + c] = xn;
      if (DOT && dot) acc += (double)S[ro + c] * (double)xn;
    }
    __syncthreads();
    flip ^= 1u << l;
  };
  // down: pre-smoothing (from zero) and restriction rc = (1/8) sum_children (r - A x)
  for (int l = 0; l < L - 1; ++l) {
    for (int t = 0; t < TL.nu[l]; ++t) sweep(l, t == 0, false);
    const int nx = TL.nx[l], ny = TL.ny[l], nz = TL.nz[l], sx = ny * nz;
    const int CY = TL.ny[l + 1], CZ = TL.nz[l + 1], nc = TL.nx[l + 1] * CY * CZ;
    const int ro = Ro(l), xo = Xo(l), qo = Qo(l), dg = Do(l), rc = Ro(l + 1);
    const T sc = TL.sc[l];
    for (int cc = threadIdx.x; cc < nc; cc += TAIL_BLOCK) {
      int I, J, K;
      decl(l + 1, cc, I, J, K);
      T sres = 0;
      for (int di = 0; di < 2; ++di)
        for (int dj = 0; dj < 2; ++dj)
          for (int dk = 0; dk < 2; ++dk) {
            const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
            if (i < nx && j < ny && k < nz) {
              const int f = (i * ny + j) * nz + k;
              const T q = S[qo + f];
              T off = 0;
              if (i > 0) off += (q + S[qo + f - sx]) * S[xo + f - sx];
              if (i < nx - 1) off += (q + S[qo + f + sx]) * S[xo + f + sx];
              if (j > 0) off += (q + S[qo + f - nz]) * S[xo + f - nz];
              if (j < ny - 1) off += (q + S[qo + f + nz]) * S[xo + f + nz];
              if (k > 0) off += (q + S[qo + f - 1]) * S[xo + f - 1];
              if (k < nz - 1) off += (q + S[qo + f + 1]) * S[xo + f + 1];
              sres += S[ro + f] - (S[xo + f] / S[dg + f] - T(0.5) * sc * off);
            }
          }
      S[rc + cc] = T(0.125) * sres;
    }
    __syncthreads();
  }
  // coarsest level
  for (int t = 0; t < coarse_sweeps; ++t) sweep(L - 1, t == 0, L == 1 && t == coarse_sweeps - 1);
  // up: injection of the coarse correction, then post-smoothing
  for (int l = L - 2; l >= 0; --l) {
    const int nx = TL.nx[l], ny = TL.ny[l], nz = TL.nz[l], n = nx * ny * nz;
    const int CY = TL.ny[l + 1], CZ = TL.nz[l + 1], xo = Xo(l), xc = Xo(l + 1);
    for (int c = threadIdx.x; c < n; c += TAIL_BLOCK) {
      int i, j, k;
      decl(l, c, i, j, k);
      S[xo + c] += S[xc + ((i >> 1) * CY + (j >> 1)) * CZ + (k >> 1)];
    }
    __syncthreads();
    for (int t = 0; t < TL.nu[l]; ++t) sweep(l, false, l == 0 && t == TL.nu[l] - 1);
  }
  const int x0 = Xo(0);
  for (int c = threadIdx.x; c < N(0); c += TAIL_BLOCK) xout[c] = S[x0 + c];
  if (DOT) {
    __shared__ double red[TAIL_BLOCK / 64];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < TAIL_BLOCK / 64; ++w) t += red[w];
      if (!first) st->beta = t / st->rz;
      st->rz = t;
    }
  }
}

// Approximately solve A_l x = r from x = 0; the buffer holding x is returned in *out.
template <class T>
static void mg_vcycle(MgHier<T>& H, int l, const T* r, SolveStatus* st, double* partials, unsigned* counter,
                      bool dot_first, bool dot, hipStream_t s, T** out) {
  const Lev<T>& L = H.lev[l];
  const T om = (T)H.omega;
  T* a = H.x[l];
  T* b = H.t[l];
  const bool vec = use_vec(L);
  const int nb = vec ? vec_blocks(vec_items(L)) : tile_blocks(L.ntiles);
  const Lev<T> M = vec ? march_lev(L, 1) : L;   // the marching kernels' view and grid
  const int nbm = vec ? march_blocks(M) : nb;
  const bool coarsest = (l == H.nlev - 1);
  const int nu = l == 0 ? H.nu_fine : H.nu;
  const int pre = coarsest ? std::max(2, H.coarse_sweeps) : nu;
  const size_t tb = tail_bytes(H, l);
  if (H.tail && tb <= TAIL_LDS_MAX) {
    TailLevs<T> TL{};
    TL.nlev = H.nlev - l;
    int o = 0;
    for (int m = 0; m < TL.nlev; ++m) {
      const Lev<T>& Lm = H.lev[l + m];
      TL.off[m] = o;
      o += 5 * (int)Lm.n;
      TL.nx[m] = Lm.nx;
      TL.ny[m] = Lm.ny;
      TL.nz[m] = Lm.nz;
      const bool p2 = (Lm.ny & (Lm.ny - 1)) == 0 && (Lm.nz & (Lm.nz - 1)) == 0;
      TL.ly[m] = p2 ? __builtin_ctz((unsigned)Lm.ny) : -1;
      TL.lz[m] = p2 ? __builtin_ctz((unsigned)Lm.nz) : -1;
      TL.nu[m] = l + m == 0 ? H.nu_fine : H.nu;
      TL.sc[m] = Lm.sc;
      TL.q[m] = Lm.qc;
      TL.d[m] = Lm.diag;
    }
    static bool attr_set[2] = {false, false};
    auto kt = dot ? k_mg_tail<T, true> : k_mg_tail<T, false>;
    if (!attr_set[dot ? 1 : 0]) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(kt), hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)TAIL_LDS_MAX);
      attr_set[dot ? 1 : 0] = true;
    }
    kt<<<1, TAIL_BLOCK, tb, s>>>(TL, r, a, om, std::max(2, H.coarse_sweeps), st, dot_first ? 1 : 0);
    *out = a;
    return;
  }
  auto smooth = [&](bool d, int df) {
    if (vec) {
      with_nt(M.mnt, [&](auto C) {
        constexpr int NT = decltype(C)::value;
        if (d) k_mg_smooth_v<T, true, NT><<<nbm, NT, 0, s>>>(M, r, a, b, om, st, partials, counter, df);
        else k_mg_smooth_v<T, false, NT><<<nbm, NT, 0, s>>>(M, r, a, b, om, st, partials, counter, 0);
      });
    } else {
      if (d) k_mg_smooth<T, true><<<nb, BLOCK, 0, s>>>(L, r, a, b, om, st, partials, counter, df);
      else k_mg_smooth<T, false><<<nb, BLOCK, 0, s>>>(L, r, a, b, om, st, partials, counter, 0);
    }
  };
  const Lev<T> Mr = vec ? march_lev(L, 1, H.rb_threads) : L;   // the coloured sweeps' view and grid
  if (vec && H.rb && !coarsest && rb_marching_ok(Mr, H.rb_min_planes)) {
    // coloured sweeps: pre-smoothing from x = 0 relaxing the even colour
    // first, post-smoothing (the first with the prolongation) the odd one
    const int nr = H.nu_rb;
    const int nbr = march_blocks(Mr);
    const T w = (T)H.w_rb;
    const Lev<T>& C = H.lev[l + 1];
    auto rb = [&](int mode, bool d, const T* xin, const T* xcs, T* xo, int c0) {
      if constexpr (std::is_same<T, float>::value) {
        auto go = [&](auto WEc, auto CQc) {
          constexpr bool WE = decltype(WEc)::value;
          constexpr bool CQ = decltype(CQc)::value;
          with_nt(Mr.mnt, [&](auto K) {
            constexpr int NT = decltype(K)::value;
            if (mode == RB_ZERO)
              k_mg_rb_v<T, RB_ZERO, false, NT, WE, CQ><<<nbr, NT, 0, s>>>(Mr, C, r, nullptr, nullptr, xo, w, c0, st,
                                                                      partials, counter, 0);
            else if (mode == RB_PROLONG && d)
              k_mg_rb_v<T, RB_PROLONG, true, NT, WE, CQ><<<nbr, NT, 0, s>>>(Mr, C, r, xin, xcs, xo, w, c0, st, partials,
                                                                        counter, dot_first);
            else if (mode == RB_PROLONG)
              k_mg_rb_v<T, RB_PROLONG, false, NT, WE, CQ><<<nbr, NT, 0, s>>>(Mr, C, r, xin, xcs, xo, w, c0, st,
                                                                         partials, counter, 0);
            else if (d)
              k_mg_rb_v<T, RB_GEN, true, NT, WE, CQ><<<nbr, NT, 0, s>>>(Mr, C, r, xin, nullptr, xo, w, c0, st, partials,
                                                                    counter, dot_first);
            else
              k_mg_rb_v<T, RB_GEN, false, NT, WE, CQ><<<nbr, NT, 0, s>>>(Mr, C, r, xin, nullptr, xo, w, c0, st,
                                                                         partials, counter, 0);
          });
        };
        if (rows_cross_waves(Mr)) go(std::true_type{}, std::false_type{});
        else if (Mr.qk != T(0)) go(std::false_type{}, std::true_type{});   // a constant-coefficient level
        else go(std::false_type{}, std::false_type{});
      }
    };
    rb(RB_ZERO, false, nullptr, nullptr, a, 0);
    for (int t = 1; t < nr; ++t) {
      rb(RB_GEN, false, a, nullptr, b, 0);
      std::swap(a, b);
    }
    if (restrict_marching_ok(L)) {
      const Lev<T> Mp = march_lev_pairs(L);
      with_nt(Mp.mnt, [&](auto K) {
        constexpr int NT = decltype(K)::value;
        k_mg_restrict_m<T, NT><<<march_blocks(Mp), NT, 0, s>>>(Mp, C, r, a, H.r[l + 1], st);
      });
    } else {
      Lev<T> G = C;
      G.nz = L.nz;
      k_mg_restrict_v<T><<<vec_blocks(vec_items(G)), BLOCK, 0, s>>>(L, C, r, a, H.r[l + 1], st);
    }
    T* xc = nullptr;
    mg_vcycle(H, l + 1, H.r[l + 1], st, partials, counter, false, false, s, &xc);
    for (int t = 0; t < nr; ++t) {
      rb(t == 0 ? RB_PROLONG : RB_GEN, dot && t == nr - 1, a, xc, b, 1);
      std::swap(a, b);
    }
    *out = a;
    return;
  }
  if (coarsest && L.n <= COARSE_MAX) {
    if (dot) k_mg_coarse<T, true><<<1, BLOCK, 0, s>>>(L, r, a, om, pre, st, partials, counter, dot_first);
    else k_mg_coarse<T, false><<<1, BLOCK, 0, s>>>(L, r, a, om, pre, st, partials, counter, 0);
    *out = a;
    return;
  }
  int t0 = 1;
  if (vec && pre >= 2 && !(coarsest && dot && pre == 2)) {
    with_nt(M.mnt, [&](auto C) {
      constexpr int NT = decltype(C)::value;
      k_mg_smooth_two_v<T, NT><<<nbm, NT, 0, s>>>(M, r, a, om, st);
    });
    t0 = 2;
  } else if (vec) {
    k_mg_smooth_zero_v<T><<<nb, BLOCK, 0, s>>>(L, r, a, om, st);
  } else {
    k_mg_smooth_zero<T><<<nb, BLOCK, 0, s>>>(L, r, a, om, st);
  }
  for (int t = t0; t < pre; ++t) {
    smooth(coarsest && dot && t == pre - 1, dot_first);
    std::swap(a, b);
  }
  if (coarsest) {
    *out = a;
    return;
  }
  const Lev<T>& C = H.lev[l + 1];
  if (vec && restrict_marching_ok(L)) {
    const Lev<T> Mp = march_lev_pairs(L);
    with_nt(Mp.mnt, [&](auto K) {
      constexpr int NT = decltype(K)::value;
      k_mg_restrict_m<T, NT><<<march_blocks(Mp), NT, 0, s>>>(Mp, C, r, a, H.r[l + 1], st);
    });
  } else if (vec) {
    Lev<T> G = C;
    G.nz = L.nz;
    k_mg_restrict_v<T><<<vec_blocks(vec_items(G)), BLOCK, 0, s>>>(L, C, r, a, H.r[l + 1], st);
  } else {
    k_mg_restrict<T><<<tile_blocks(C.ntiles), BLOCK, 0, s>>>(L, C, r, a, H.r[l + 1], st);
  }
  T* xc = nullptr;
  mg_vcycle(H, l + 1, H.r[l + 1], st, partials, counter, false, false, s, &xc);
  for (int t = 0; t < nu; ++t) {
    const bool d = dot && t == nu - 1;
    if (t == 0) {
      if (vec) {
        with_nt(M.mnt, [&](auto K) {
          constexpr int NT = decltype(K)::value;
          if (d)
            k_mg_prolong_smooth_v<T, true, NT><<<nbm, NT, 0, s>>>(M, C, r, a, xc, b, om, st, partials, counter,
                                                                 dot_first);
          else k_mg_prolong_smooth_v<T, false, NT><<<nbm, NT, 0, s>>>(M, C, r, a, xc, b, om, st, partials, counter, 0);
        });
      } else {
        if (d) k_mg_prolong_smooth<T, true><<<nb, BLOCK, 0, s>>>(L, C, r, a, xc, b, om, st, partials, counter, dot_first);
        else k_mg_prolong_smooth<T, false><<<nb, BLOCK, 0, s>>>(L, C, r, a, xc, b, om, st, partials, counter, 0);
      }
    } else {
      smooth(d, dot_first);
    }
    std::swap(a, b);
  }
  *out = a;
}

template <class T>
void launch_neumann_start(const Lev<T>& L, const T* r, T* z, SolveStatus* st, double* partials, unsigned* counter,
                          hipStream_t s) {
  const Lev<T> M = march_lev(L);
  with_nt(M.mnt, [&](auto K) {
    constexpr int NT = decltype(K)::value;
    k_cg_update_neu_v<T, true, NT><<<march_blocks(M), NT, 0, s>>>(M, r, nullptr, nullptr, z, st, partials, counter);
  });
}
template void launch_neumann_start<double>(const Lev<double>&, const double*, double*, SolveStatus*, double*,
                                           unsigned*, hipStream_t);
template void launch_neumann_start<float>(const Lev<float>&, const float*, float*, SolveStatus*, double*, unsigned*,
                                          hipStream_t);

template <class T>
void cg_start(const Lev<T>& L, MgHier<T>* H, CgVecs<T>& V, T** z, SolveStatus* st, double* partials,
              unsigned* counters, hipStream_t s) {
  const int first = 1;
  if (H) {
    mg_vcycle(*H, 0, V.r, st, partials, counters + 2, first != 0, true, s, z);
  } else {
    *z = nullptr;
    if (use_vec(L) && V.zj && V.r_alt)
      launch_neumann_start(L, V.r, V.zj, st, partials, counters + 2, s);
    else if (use_vec(L))
      k_jac_rz_v<T><<<vec_blocks(vec_items(L)), BLOCK, 0, s>>>(L, V.r, st, partials, counters + 2, first, V.zj);
    else k_jac_rz<T><<<tile_blocks(L.ntiles), BLOCK, 0, s>>>(L, V.r, st, partials, counters + 2, first);
  }
}

template <class T>
void cg_iteration(const Lev<T>& L, MgHier<T>* H, CgVecs<T>& V, T** z, SolveStatus* st, double* partials,
                  unsigned* counters, bool first, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  const bool vec = use_vec(L);
  const int nb = vec ? vec_blocks(vec_items(L)) : tile_blocks(L.ntiles);
  const Lev<T> M = vec ? march_lev(L) : L;   // the operator kernel's view and grid
  const int nbm = vec ? march_blocks(M) : nb;
  // vectorised levels defer x += alpha p into the next direction update
  T* xd = vec ? V.x : nullptr;
  if (H) {
    if (vec) {
      with_nt(M.mnt, [&](auto K) {
        constexpr int NT = decltype(K)::value;
        auto kdir = dir_v<T, false, NT>(first);
        if (ev0) {
          // events attached to the dispatch itself: kernel start and end times
          hipExtLaunchKernelGGL(kdir, dim3(nbm), dim3(NT), 0, s, ev0, ev1, 0, M, (const T*)*z, (const T*)V.r,
                                (const T*)V.p, V.p_alt, V.q, st, partials, counters, xd);
        } else {
          kdir<<<nbm, NT, 0, s>>>(M, *z, V.r, V.p, V.p_alt, V.q, st, partials, counters, xd);
        }
      });
    } else {
      auto kdir = k_cg_dir_spmv<T, false>;
      if (ev0)
        hipExtLaunchKernelGGL(kdir, dim3(nb), dim3(BLOCK), 0, s, ev0, ev1, 0, L, (const T*)*z, (const T*)V.r,
                              (const T*)V.p, V.p_alt, V.q, st, partials, counters, (int)first);
      else
        kdir<<<nb, BLOCK, 0, s>>>(L, *z, V.r, V.p, V.p_alt, V.q, st, partials, counters, first);
    }
    std::swap(V.p, V.p_alt);
    if (vec) k_cg_update_v<T, false><<<nb, BLOCK, 0, s>>>(L, nullptr, V.r, V.p, V.q, st, partials, counters + 1, nullptr);
    else k_cg_update<T, false><<<nb, BLOCK, 0, s>>>(L, V.x, V.r, V.p, V.q, st, partials, counters + 1);
    mg_vcycle(*H, 0, V.r, st, partials, counters + 2, false, true, s, z);
  } else {
    if (vec && V.zj) {
      // z = M^-1 r was stored by the previous update (or the start)
      with_nt(M.mnt, [&](auto K) {
        constexpr int NT = decltype(K)::value;
        dir_v<T, false, NT>(first)<<<nbm, NT, 0, s>>>(M, V.zj, V.r, V.p, V.p_alt, V.q, st, partials, counters, xd);
      });
      std::swap(V.p, V.p_alt);
      if (V.r_alt) {
        // Neumann-polynomial z; r' into the second buffer
        with_nt(M.mnt, [&](auto K) {
          constexpr int NT = decltype(K)::value;
          k_cg_update_neu_v<T, false, NT><<<nbm, NT, 0, s>>>(M, V.r, V.r_alt, V.q, V.zj, st, partials,
                                                              counters + 1);
        });
        std::swap(V.r, V.r_alt);
      } else {
        k_cg_update_v<T, true><<<nb, BLOCK, 0, s>>>(L, nullptr, V.r, V.p, V.q, st, partials, counters + 1, V.zj);
      }
    } else if (vec) {
      with_nt(M.mnt, [&](auto K) {
        constexpr int NT = decltype(K)::value;
        dir_v<T, true, NT>(first)<<<nbm, NT, 0, s>>>(M, nullptr, V.r, V.p, V.p_alt, V.q, st, partials, counters, xd);
      });
      std::swap(V.p, V.p_alt);
      k_cg_update_v<T, true><<<nb, BLOCK, 0, s>>>(L, nullptr, V.r, V.p, V.q, st, partials, counters + 1, nullptr);
    } else {
      k_cg_dir_spmv<T, true><<<nb, BLOCK, 0, s>>>(L, nullptr, V.r, V.p, V.p_alt, V.q, st, partials, counters, first);
      std::swap(V.p, V.p_alt);
      k_cg_update<T, true><<<nb, BLOCK, 0, s>>>(L, V.x, V.r, V.p, V.q, st, partials, counters + 1);
    }
  }
}

template <class T>
bool cg_defers_x(const Lev<T>& L) {
  return use_vec(L);
}
template bool cg_defers_x<double>(const Lev<double>&);
template bool cg_defers_x<float>(const Lev<float>&);

// Back-to-back launches of the multigrid CG operator kernel (direction
// update with beta from st, matrix-free product, <p, q>) between two events;
// returns the mean duration in microseconds.  Same kernel and launch shape
// as inside the pressure solve.
template <class T>
double replay_operator_kernel(const Lev<T>& L, const T* z, const T* pin, T* pout, T* q, SolveStatus* st,
                              double* partials, unsigned* counter, int reps, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1) {
  const bool vec = use_vec(L);
  const Lev<T> M = vec ? march_lev(L) : L;
  const int nb = vec ? march_blocks(M) : tile_blocks(L.ntiles);
  auto launch = [&]() {
    if (vec) {
      with_nt(M.mnt, [&](auto K) {
        constexpr int NT = decltype(K)::value;
        k_cg_dir_spmv_v<T, false, false, NT><<<nb, NT, 0, s>>>(M, z, nullptr, pin, pout, q, st, partials, counter,
                                                               nullptr);
      });
    } else {
      k_cg_dir_spmv<T, false><<<nb, BLOCK, 0, s>>>(M, z, nullptr, pin, pout, q, st, partials, counter, 0);
    }
  };
  launch();
  if (hipEventRecord(e0, s) != hipSuccess) return -1.0;
  for (int t = 0; t < reps; ++t) launch();
  if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
  return 1e3 * (double)ms / reps;
}
// Back-to-back launches of the fine level's smoother sweep as the V-cycle of
// hierarchy H runs it there (a coloured sweep from x where the level takes
// them, else damped Jacobi) between two events; mean duration in microseconds.
template <class T>
double replay_smooth_kernel(const Lev<T>& L, const MgHier<T>& H, const T* r, const T* xin, T* xout, SolveStatus* st,
                            int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
  const bool vec = use_vec(L);
  const Lev<T> M = vec ? march_lev(L, 1) : L;
  const int nb = vec ? march_blocks(M) : tile_blocks(L.ntiles);
  const double omega = H.omega;
  const Lev<T> Mr = vec ? march_lev(L, 1, H.rb_threads) : L;
  const bool rb = vec && H.rb && rb_marching_ok(Mr, H.rb_min_planes);
  const int nbr = rb ? march_blocks(Mr) : 0;
  auto launch = [&]() {
    if (rb) {
      if constexpr (std::is_same<T, float>::value) {
        auto go = [&](auto WEc) {
          constexpr bool WE = decltype(WEc)::value;
          with_nt(Mr.mnt, [&](auto K) {
            constexpr int NT = decltype(K)::value;
            k_mg_rb_v<T, RB_GEN, false, NT, WE><<<nbr, NT, 0, s>>>(Mr, Mr, r, xin, nullptr, xout, (T)H.w_rb, 0, st,
                                                                   nullptr, nullptr, 0);
          });
        };
        if (rows_cross_waves(Mr)) go(std::true_type{});
        else go(std::false_type{});
      }
    } else if (vec) {
      with_nt(M.mnt, [&](auto K) {
        constexpr int NT = decltype(K)::value;
        k_mg_smooth_v<T, false, NT><<<nb, NT, 0, s>>>(M, r, xin, xout, (T)omega, st, nullptr, nullptr, 0);
      });
    } else {
      k_mg_smooth<T, false><<<nb, BLOCK, 0, s>>>(M, r, xin, xout, (T)omega, st, nullptr, nullptr, 0);
    }
  };
  launch();
  if (hipEventRecord(e0, s) != hipSuccess) return -1.0;
  for (int t = 0; t < reps; ++t) launch();
  if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
  return 1e3 * (double)ms / reps;
}
template double replay_smooth_kernel<double>(const Lev<double>&, const MgHier<double>&, const double*, const double*,
                                             double*, SolveStatus*, int, hipStream_t, hipEvent_t, hipEvent_t);
template double replay_smooth_kernel<float>(const Lev<float>&, const MgHier<float>&, const float*, const float*, float*,
                                            SolveStatus*, int, hipStream_t, hipEvent_t, hipEvent_t);

template double replay_operator_kernel<double>(const Lev<double>&, const double*, const double*, double*, double*,
                                               SolveStatus*, double*, unsigned*, int, hipStream_t, hipEvent_t,
                                               hipEvent_t);
template double replay_operator_kernel<float>(const Lev<float>&, const float*, const float*, float*, float*,
                                              SolveStatus*, double*, unsigned*, int, hipStream_t, hipEvent_t,
                                              hipEvent_t);

bool resid64_cq_ok(const Lev<double>& L) { return use_vec(L); }
void launch_resid64(const Lev<double>& L, const double* b, const double* x, double* r, SolveStatus* st,
                    double* partials, unsigned* counter, bool set_bnorm, hipStream_t s, float* r32, bool cq) {
  if (use_vec(L)) {
    const Lev<double> M = march_lev(L);
    with_nt(M.mnt, [&](auto K) {
      constexpr int NT = decltype(K)::value;
      if (cq && M.qk != 0.0)
        k_resid64_v<NT, true><<<march_blocks(M), NT, 0, s>>>(M, b, x, r, st, partials, counter, set_bnorm ? 1 : 0,
                                                             r32);
      else
        k_resid64_v<NT><<<march_blocks(M), NT, 0, s>>>(M, b, x, r, st, partials, counter, set_bnorm ? 1 : 0, r32);
    });
  } else {
    k_resid64<<<tile_blocks(L.ntiles), BLOCK, 0, s>>>(L, b, x, r, st, partials, counter, set_bnorm ? 1 : 0);
    if (r32) k_to_float<<<grid_blocks(L.n), BLOCK, 0, s>>>(r, r32, L.n);
  }
}
void launch_zero_if_flagged(double* x, long long n, const SolveStatus* st, hipStream_t s, double* r) {
  k_zero_if_flagged<<<grid_blocks(n), BLOCK, 0, s>>>(x, r, n, st);
}
template <class T>
void launch_inner_init(const Lev<T>& L, const double* r64, T* r, T* x, SolveStatus* st, double* partials,
                       unsigned* counter, hipStream_t s) {
  if (use_vec(L)) k_inner_init_v<T><<<vec_blocks(vec_items(L)), BLOCK, 0, s>>>(L, r64, r, x, st, partials, counter);
  else k_inner_init<T><<<tile_blocks(L.ntiles), BLOCK, 0, s>>>(L, r64, r, x, st, partials, counter);
}
template <class T>
void launch_add_correction(const Lev<T>& L, double* x, const T* e, hipStream_t s, const T* p,
                           const SolveStatus* st) {
  if (use_vec(L)) {
    k_add_correction_v<T><<<vec_blocks(vec_items(L)), BLOCK, 0, s>>>(L, x, e, p, st, nullptr);
  } else {
    if (p) launch_axpy_alpha<T>(const_cast<T*>(e), p, st, L.n, s);
    k_add_correction<T><<<tile_blocks(L.ntiles), BLOCK, 0, s>>>(L, x, e);
  }
}
template <class T>
bool launch_inner_init_jac(const Lev<T>& L, const double* r64, T* r, T* x, T* z, SolveStatus* st, double* partials,
                           unsigned* counter, hipStream_t s) {
  if (!use_vec(L)) return false;
  k_inner_init_jac_v<T><<<vec_blocks(vec_items(L)), BLOCK, 0, s>>>(L, r64, r, x, z, st, partials, counter);
  return true;
}
template bool launch_inner_init_jac<float>(const Lev<float>&, const double*, float*, float*, float*, SolveStatus*,
                                           double*, unsigned*, hipStream_t);
void launch_add_correction_by_parity(const Lev<float>& L, double* x, const float* e, const float* p_even,
                                     const float* p_odd, const SolveStatus* st, hipStream_t s) {
  k_add_correction_v<float><<<vec_blocks(vec_items(L)), BLOCK, 0, s>>>(L, x, e, p_even, st, p_odd);
}
void launch_to_float(const double* a, float* b, long long n, hipStream_t s) {
  k_to_float<<<grid_blocks(n), BLOCK, 0, s>>>(a, b, n);
}

// A fresh solve status (zeros, tol, maxit) written on the device: stream
// ordered without a host-to-device copy, which from pageable memory would be
// staged by the runtime.
__global__ void k_init_status(SolveStatus* __restrict__ st, double tol, int maxit) {
  if (threadIdx.x == 0) {
    SolveStatus v{};
    v.tol = tol;
    v.maxit = maxit;
    *st = v;
  }
}
void launch_init_status(SolveStatus* st, double tol, int maxit, hipStream_t s) {
  k_init_status<<<1, 64, 0, s>>>(st, tol, maxit);
}

// An inner solve's fresh status whose tolerance is the reduction the outer
// solve still needs: min(hi, max(lo, num / outer res)).
__global__ void k_init_inner_status(SolveStatus* __restrict__ st, const SolveStatus* __restrict__ outer, double num,
                                    double lo, double hi, int maxit) {
  if (threadIdx.x == 0) {
    SolveStatus v{};
    v.tol = fmin(hi, fmax(lo, num / fmax(outer->res, 1e-300)));
    v.maxit = maxit;
    *st = v;
  }
}
void launch_init_inner_status(SolveStatus* st, const SolveStatus* outer, double num, double lo, double hi, int maxit,
                              hipStream_t s) {
  k_init_inner_status<<<1, 64, 0, s>>>(st, outer, num, lo, hi, maxit);
}

// FP64 CG preconditioned by the FP32 V-cycle (levels whose nz is even).
void cg_start_mg32(const Lev<double>& L, MgHier<float>& H, const double* r64, float* r32, float** z, SolveStatus* st,
                   double* partials, unsigned* counters, hipStream_t s, bool r32_ready) {
  if (!r32_ready) k_to_float<<<grid_blocks(L.n), BLOCK, 0, s>>>(r64, r32, L.n);
  mg_vcycle(H, 0, r32, st, partials, counters + 2, true, true, s, z);
}
void cg_iteration_mg32(const Lev<double>& L, MgHier<float>& H, CgVecsMg32& V, float* r32, float** z,
                       SolveStatus* st, double* partials, unsigned* counters, bool first, hipStream_t s) {
  const int nb = vec_blocks(vec_items(L));
  const Lev<double> M = march_lev(L);
  const int nbm = march_blocks(M);
  with_nt(M.mnt, [&](auto K) {
    constexpr int NT = decltype(K)::value;
    // a constant-coefficient system (M.qk set) takes q from a register
    if (first && M.qk != 0.0)
      k_cg_dir_spmv_z32_v<true, NT, true><<<nbm, NT, 0, s>>>(M, *z, V.p, V.p_alt, V.q, st, partials, counters, V.x);
    else if (first)
      k_cg_dir_spmv_z32_v<true, NT><<<nbm, NT, 0, s>>>(M, *z, V.p, V.p_alt, V.q, st, partials, counters, V.x);
    else if (M.qk != 0.0)
      k_cg_dir_spmv_z32_v<false, NT, true><<<nbm, NT, 0, s>>>(M, *z, V.p, V.p_alt, V.q, st, partials, counters, V.x);
    else
      k_cg_dir_spmv_z32_v<false, NT><<<nbm, NT, 0, s>>>(M, *z, V.p, V.p_alt, V.q, st, partials, counters, V.x);
  });
  std::swap(V.p, V.p_alt);
  k_cg_update_r32_v<<<nb, BLOCK, 0, s>>>(L, V.r, V.q, r32, st, partials, counters + 1);
  mg_vcycle(H, 0, r32, st, partials, counters + 2, false, true, s, z);
}
bool mg32_supported(const Lev<double>& L) { return use_vec(L); }
// Two non-first iterations of that CG recorded on the capture stream cs into
// an executable graph (null if capture or instantiation fails).  Replaying it
// advances the solve by two iterations: the direction buffers swap twice, so
// the pointers the graph holds are those of the next pair again, and the
// V-cycle's output buffer z is the same every iteration.  Every kernel reads
// alpha, beta and the converged flag from the device status, so a replay
// after convergence does no work.
hipGraphExec_t capture_mg32_pair(const Lev<double>& L, MgHier<float>& H, CgVecsMg32 V, float* r32, float* z,
                                 SolveStatus* st, double* partials, unsigned* counters, hipStream_t cs) {
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeRelaxed) != hipSuccess) return nullptr;
  cg_iteration_mg32(L, H, V, r32, &z, st, partials, counters, false, cs);
  cg_iteration_mg32(L, H, V, r32, &z, st, partials, counters, false, cs);
  hipGraph_t gr = nullptr;
  if (hipStreamEndCapture(cs, &gr) != hipSuccess || !gr) {
    (void)hipGetLastError();
    return nullptr;
  }
  hipGraphExec_t ex = nullptr;
  const hipError_t e = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    return nullptr;
  }
  return ex;
}
double replay_operator_z32(const Lev<double>& L, const float* z, const float* pin, float* pout, double* q,
                           SolveStatus* st, double* partials, unsigned* counter, int reps, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1) {
  const Lev<double> M = march_lev(L);
  const int nb = march_blocks(M);
  auto launch = [&]() {
    with_nt(M.mnt, [&](auto K) {
      constexpr int NT = decltype(K)::value;
      k_cg_dir_spmv_z32_v<false, NT><<<nb, NT, 0, s>>>(M, z, pin, pout, q, st, partials, counter, nullptr);
    });
  };
  launch();
  if (hipEventRecord(e0, s) != hipSuccess) return -1.0;
  for (int t = 0; t < reps; ++t) launch();
  if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) return -1.0;
  float ms = 0.f;
  if (hipEventElapsedTime(&ms, e0, e1) != hipSuccess) return -1.0;
  return 1e3 * (double)ms / reps;
}

template <class T>
void launch_mg_diag(const Lev<T>& L, int dirmask, T* dout, hipStream_t s) {
  k_mg_diag<T><<<tile_blocks(L.ntiles), BLOCK, 0, s>>>(L, dirmask, dout);
}
template void launch_mg_diag<float>(const Lev<float>&, int, float*, hipStream_t);
template void mg_setup_levels<double>(MgHier<double>&, int, hipStream_t);
template void mg_setup_levels<float>(MgHier<float>&, int, hipStream_t);
template void cg_start<double>(const Lev<double>&, MgHier<double>*, CgVecs<double>&, double**, SolveStatus*,
                               double*, unsigned*, hipStream_t);
template void cg_start<float>(const Lev<float>&, MgHier<float>*, CgVecs<float>&, float**, SolveStatus*, double*,
                              unsigned*, hipStream_t);
template void cg_iteration<double>(const Lev<double>&, MgHier<double>*, CgVecs<double>&, double**, SolveStatus*,
                                   double*, unsigned*, bool, hipStream_t, hipEvent_t, hipEvent_t);
template void cg_iteration<float>(const Lev<float>&, MgHier<float>*, CgVecs<float>&, float**, SolveStatus*,
                                  double*, unsigned*, bool, hipStream_t, hipEvent_t, hipEvent_t);
template void launch_inner_init<float>(const Lev<float>&, const double*, float*, float*, SolveStatus*, double*,
                                       unsigned*, hipStream_t);
template void launch_add_correction<float>(const Lev<float>&, double*, const float*, hipStream_t, const float*,
                                          const SolveStatus*);

}  // namespace dsv
