// Level descriptors, tile mapping and launchers of the conjugate-gradient
// solvers (Jacobi or geometric multigrid preconditioning, FP64 or FP32).
#pragma once
#include <hip/hip_runtime.h>

#include <utility>

#include "ds_device.h"

namespace dsv {

constexpr int MG_MAXLEV = 12;
constexpr int TK = 64;   // tile extent along z (one wavefront)
constexpr int TJ = 4;    // tile extent along y (four wavefronts per block)

// One level's operator: (A x)_c = diag_c x_c - sc/2 sum_nb (q_c + q_nb) x_nb,
// plus its 64x4 tile decomposition.
// Launch shapes of the solver kernels.  Each handle holds its own; the entry
// points of the library make the calling handle's shape current on the
// calling thread (ShapeScope) before they build levels or launch kernels.
struct LaunchShape {
  // Rows of y per slab in the item order of the z-vectorised kernels: items
  // run z-fastest, then y within a slab of `ytile` rows, then x, then slab.
  // Neighbours in x are then one slab-plane apart instead of a full plane,
  // which keeps the x-1, x, x+1 working set of a streaming pass inside one
  // XCD's L2.  0 or a value not dividing ny: whole planes.
  int vec_ytile = 0;
  int vec_max_blocks = 1024;   // grid cap of the z-vectorised pointwise kernels
  int march_threads = 262144;  // threads (columns x chunks) the marching kernels aim for
  int march_min_planes = 1;    // shortest chunk of x-planes a marching thread walks
  // block sizes (256, 384, 512) the marching kernels of class 0 (CG operator,
  // FP64 residual) and class 1 (V-cycle sweeps, restriction) try in order
  int march_pref[2][4] = {{512, 256, 384, 0}, {256, 512, 384, 0}};
};
// The calling thread's current shape (the defaults outside any scope).
const LaunchShape& launch_shape();
class ShapeScope {
 public:
  explicit ShapeScope(const LaunchShape* s);
  ~ShapeScope();
  ShapeScope(const ShapeScope&) = delete;
  ShapeScope& operator=(const ShapeScope&) = delete;

 private:
  const LaunchShape* prev_;
};

template <class T>
struct Lev {
  int nx, ny, nz;
  int ytile;
  int mch;     // chunks of x-planes per column in the marching kernels (set by the launcher)
  int mnt;     // threads per block of the marching kernels (set by the launcher)
  int dfly;    // 1: the marching kernels form diag from qc (pressure-type operator) instead of loading it
  int dmask;   // with dfly: bit (axis*2 + side) set where the box face is p = 0 (Dirichlet)
  T qk;        // nonzero: qc holds this value in every cell (the coloured sweep then loads no q)
  int ntk, ntj;
  unsigned ntiles;
  long long n;
  T sc;
  const T* qc;
  const T* diag;
};

template <class T>
inline void lev_dims(Lev<T>& L, int nx, int ny, int nz, double sc) {
  L.nx = nx;
  L.ny = ny;
  L.nz = nz;
  const int yt = launch_shape().vec_ytile;
  L.ytile = (yt > 0 && ny % yt == 0) ? yt : ny;
  L.mch = 1;
  L.mnt = 256;
  L.dfly = 0;
  L.dmask = 0;
  L.qk = 0;
  L.ntk = (nz + TK - 1) / TK;
  L.ntj = (ny + TJ - 1) / TJ;
  L.ntiles = (unsigned)L.ntk * (unsigned)L.ntj * (unsigned)nx;
  L.n = (long long)nx * ny * nz;
  L.sc = (T)sc;
}

template <class T>
struct MgHier {
  int nlev = 0;
  Lev<T> lev[MG_MAXLEV];
  T* r[MG_MAXLEV] = {};   // level right-hand sides (level 0: the CG residual, not stored here)
  T* x[MG_MAXLEV] = {};   // level iterates (ping-pong with t)
  T* t[MG_MAXLEV] = {};
  double omega = 0.9;     // damped Jacobi weight
  int nu = 4;             // pre = post smoothing sweeps
  int nu_fine = 4;        // the same on the finest level
  int coarse_sweeps = 16; // sweeps on the coarsest level
  int tail = 1;           // run the levels that fit in one workgroup's LDS as one launch
  int rb = 1;             // coloured (x-z red-black) sweeps on the levels that allow them
  int nu_rb = 3;          // their pre = post sweeps
  double w_rb = 1.0;      // their relaxation weight
  int rb_min_planes = 8;  // shortest marching chunk a level may have to take them
  long long rb_threads = 0;   // threads their marching grid aims for (0: as the other marching kernels)
};

// CG work vectors of one precision.
template <class T>
struct CgVecs {
  T* x;        // solution (FP64 path) or correction (inner FP32 path)
  T* r;        // residual
  T* p;        // direction (ping-pong with p_alt)
  T* p_alt;
  T* q;        // A p
  T* zj = nullptr;   // Jacobi: z = r/diag stored by the update (vectorised levels)
  // with zj on vectorised levels: second residual buffer; the preconditioner is
  // then the first-order Neumann polynomial of the Jacobi splitting (the
  // diagonally dominant energy and species systems)
  T* r_alt = nullptr;
};

// Vectors of the precision form's multigrid CG: FP64 solution, residual and
// q = A p; the directions in FP32.  x and r are updated with the same
// FP32 p and q is formed from it in FP64, so the residual recurrence keeps
// FP64 accuracy.
struct CgVecsMg32 {
  double* x;
  double* r;
  float* p;
  float* p_alt;
  double* q;
};
// Two non-first iterations of the FP32-multigrid CG captured on stream cs as
// an executable graph (null on failure); z: the V-cycle output buffer.
hipGraphExec_t capture_mg32_pair(const Lev<double>& L, MgHier<float>& H, CgVecsMg32 V, float* r32, float* z,
                                 SolveStatus* st, double* partials, unsigned* counters, hipStream_t cs);
// x += st->alpha p with an FP32 p (the last deferred update of that CG).
void launch_axpy_alpha(double* x, const float* p, const SolveStatus* st, long long n, hipStream_t s);

// dirmask bit (axis*2 + side) set: p_rgh = 0 on that box face.  Every level
// (the finest included) is marked to form its diagonal from q on the fly;
// the coarse levels' stored diagonals are computed here.
template <class T>
void mg_setup_levels(MgHier<T>& H, int dirmask, hipStream_t s);
// diag of a pressure-type level from its q and the Dirichlet faces (the
// formula the marching kernels apply on the fly), into dout.
template <class T>
void launch_mg_diag(const Lev<T>& L, int dirmask, T* dout, hipStream_t s);

// Enqueue the start of a solve whose residual is already in V.r (and whose
// status holds bnorm): z = M^-1 r, rz = <r, z>.  Then iterations.
template <class T>
void cg_start(const Lev<T>& L, MgHier<T>* H, CgVecs<T>& V, T** z, SolveStatus* st, double* partials,
              unsigned* counters, hipStream_t s);
// ev0/ev1 (may be null): events recorded just before and after the operator
// kernel (direction update + matrix-free product) of a multigrid iteration.
template <class T>
void cg_iteration(const Lev<T>& L, MgHier<T>* H, CgVecs<T>& V, T** z, SolveStatus* st, double* partials,
                  unsigned* counters, bool first, hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

template <class T>
double replay_operator_kernel(const Lev<T>& L, const T* z, const T* pin, T* pout, T* q, SolveStatus* st,
                              double* partials, unsigned* counter, int reps, hipStream_t s, hipEvent_t e0,
                              hipEvent_t e1);

// The fine level's smoother sweep as the V-cycle of H runs it (coloured or
// damped Jacobi), replayed back to back; mean duration in microseconds.
template <class T>
double replay_smooth_kernel(const Lev<T>& L, const MgHier<T>& H, const T* r, const T* xin, T* xout, SolveStatus* st,
                            int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1);

// FP64 conjugate gradients preconditioned by the FP32 multigrid V-cycle
// (operator, vectors and dot products in FP64; the V-cycle's sweeps, its
// operator copies and r, z in FP32).  Needs mg32_supported(L).
bool mg32_supported(const Lev<double>& L);
// Largest grid of the z-vectorised kernels (rounded to a multiple of 8).
void set_vec_max_blocks(LaunchShape& sh, int nb);
// Threads (columns x chunks) the marching kernels aim for.
void set_march_threads(LaunchShape& sh, int n);
// Shortest chunk of x-planes a marching thread walks.
void set_march_min_planes(LaunchShape& sh, int n);
// Block sizes (256, 384, 512) the marching kernels of class cls try in order
// (0: CG operator and FP64 residual, 1: V-cycle sweeps and restriction).
void set_march_pref(LaunchShape& sh, int cls, const int* nts, int n);
double replay_operator_z32(const Lev<double>& L, const float* z, const float* pin, float* pout, double* q,
                           SolveStatus* st, double* partials, unsigned* counter, int reps, hipStream_t s, hipEvent_t e0,
                           hipEvent_t e1);
// r32_ready: r32 already holds r64 in FP32 (launch_resid64 wrote it).
void cg_start_mg32(const Lev<double>& L, MgHier<float>& H, const double* r64, float* r32, float** z, SolveStatus* st,
                   double* partials, unsigned* counters, hipStream_t s, bool r32_ready = false);
// The iteration's solution update is deferred: iteration t applies
// x += alpha_{t-1} p_{t-1}; after the last iteration t = it, launch_axpy_alpha
// with the direction buffer of that iteration applies alpha_it p_it.
void cg_iteration_mg32(const Lev<double>& L, MgHier<float>& H, CgVecsMg32& V, float* r32, float** z,
                       SolveStatus* st, double* partials, unsigned* counters, bool first, hipStream_t s);
template <class T>
void launch_axpy_alpha(T* x, const T* p, const SolveStatus* st, long long n, hipStream_t s);
// Does cg_iteration defer x += alpha p on this level (vectorised kernels)?
// Then the caller applies the last iteration's update with launch_axpy_alpha.
template <class T>
bool cg_defers_x(const Lev<T>& L);

// r = b - A x (FP64), ||b|| (if set_bnorm), ||r|| -> status (done if ||r|| <= tol ||b||).
// r32 (may be null): also store r in FP32.  r may be null where only the
// status is wanted (the marching form; see resid64_cq_ok).  cq: the operator's
// coefficient is L.qk in every cell (nonzero), taken from that value instead
// of loaded from L.qc -- the same arithmetic -- where resid64_cq_ok(L).
void launch_resid64(const Lev<double>& L, const double* b, const double* x, double* r, SolveStatus* st,
                    double* partials, unsigned* counter, bool set_bnorm, hipStream_t s, float* r32 = nullptr,
                    bool cq = false);
// Does launch_resid64 take the marching form on L (which honours cq and a null r)?
bool resid64_cq_ok(const Lev<double>& L);
// st->zero (b = 0): x = 0 and, with r, the residual r = 0 to match.
void launch_zero_if_flagged(double* x, long long n, const SolveStatus* st, hipStream_t s, double* r = nullptr);
template <class T>
void launch_inner_init(const Lev<T>& L, const double* r64, T* r, T* x, SolveStatus* st, double* partials,
                       unsigned* counter, hipStream_t s);
// x += e (FP64 x, FP32 e); with p (may be null) first e += st->alpha p.
template <class T>
void launch_add_correction(const Lev<T>& L, double* x, const T* e, hipStream_t s, const T* p = nullptr,
                           const SolveStatus* st = nullptr);
// x += e + st->alpha p with p the direction of the inner solve's last
// iteration, p_odd or p_even by the parity of st->it (read on the device;
// nothing added before the first iteration).  Vectorised levels only.
void launch_add_correction_by_parity(const Lev<float>& L, double* x, const float* e, const float* p_even,
                                     const float* p_odd, const SolveStatus* st, hipStream_t s);
// Start of a Jacobi-preconditioned round in one pass: r = (T) r64, x = 0,
// z = r/diag (z may be null: not stored), status (||r||, <r, z>).  False
// (nothing launched) off the vectorised levels.
template <class T>
bool launch_inner_init_jac(const Lev<T>& L, const double* r64, T* r, T* x, T* z, SolveStatus* st, double* partials,
                           unsigned* counter, hipStream_t s);
// First z of a Neumann-polynomial preconditioned solve (vectorised levels):
// z = (D^-1 + D^-1 N D^-1) r and st->rz = <r, z>.
template <class T>
void launch_neumann_start(const Lev<T>& L, const T* r, T* z, SolveStatus* st, double* partials, unsigned* counter,
                          hipStream_t s);
void launch_to_float(const double* a, float* b, long long n, hipStream_t s);
// *st = a fresh status (zeros, tol, maxit), written by a kernel on stream s.
void launch_init_status(SolveStatus* st, double tol, int maxit, hipStream_t s);
// *st = a fresh status with tol = min(hi, max(lo, num / outer->res)), formed
// on the device from the outer solve's residual.
void launch_init_inner_status(SolveStatus* st, const SolveStatus* outer, double num, double lo, double hi, int maxit,
                              hipStream_t s);

}  // namespace dsv
