// C-ABI of the dsvof library: handle, workspace layout and the step driver.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <utility>

#include "../../include/dsvof.h"
#include "ds_device.h"
#include "ds_kernels.h"
#include "ds_mg.h"

using namespace dsv;

namespace {

// Peng-Robinson compressibility of the pure ambient gas (largest root), host side,
// for the gas density of eq. 24.
double host_pr_Z(double T, double p, double Tc, double Pc, double om) {
  const double kap = 0.37464 + 1.54226 * om - 0.26992 * om * om;
  const double s = 1.0 + kap * (1.0 - std::sqrt(T / Tc));
  const double a = 0.45724 * R_GAS * R_GAS * Tc * Tc / Pc * s * s;
  const double b = 0.07780 * R_GAS * Tc / Pc;
  const double A = a * p / (R_GAS * T * R_GAS * T), B = b * p / (R_GAS * T);
  const double c2 = -(1.0 - B), c1 = A - 3.0 * B * B - 2.0 * B, c0 = -(A * B - B * B - B * B * B);
  double z = 1.0 + std::max(std::fabs(c2), std::max(std::fabs(c1), std::fabs(c0)));
  for (int it = 0; it < 200; ++it) {
    const double f = ((z + c2) * z + c1) * z + c0, fp = (3.0 * z + 2.0 * c2) * z + c1;
    const double dz = f / fp;
    z -= dz;
    if (std::fabs(dz) <= 1e-16 * std::fabs(z)) break;
  }
  return z;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

}  // namespace

struct ds_grid {
  ds_params prm{};
  DevParams dp{};
  long long n = 0, nu = 0, nv = 0, nw = 0;
  size_t ws_bytes = 0;
  bool bound = false;
  std::string err;
  // device arrays (carved from the workspace)
  double *alpha = nullptr, *c = nullptr, *omega = nullptr, *T = nullptr, *p = nullptr;
  double *u = nullptr, *v = nullptr, *w = nullptr;
  double *a1 = nullptr, *a_new = nullptr, *c_new = nullptr, *T_new = nullptr, *om_new = nullptr;
  double *mraw = nullptr, *mdot = nullptr, *us = nullptr, *vs = nullptr, *ws = nullptr, *xi = nullptr;
  double *b = nullptr, *r = nullptr, *pd = nullptr, *q = nullptr, *diag = nullptr, *qc = nullptr;
  int* adj = nullptr;
  double* partials = nullptr;
  unsigned* counters = nullptr;
  double* scal = nullptr;
  SolveStatus* status = nullptr;   // T, omega, p, inner FP32 solve
  double* p_alt = nullptr;         // second CG direction buffer
  double* phi = nullptr;           // potential of the divergent part of u (warm start kept)
  MgHier<double> H64;
  MgHier<float> H32;
  Lev<double> L0;                  // fine-level dimensions and tiles (operator pointers set per solve)
  float *qc32 = nullptr, *diag32 = nullptr;
  float *e32 = nullptr, *r32 = nullptr, *p32 = nullptr, *p32alt = nullptr, *q32 = nullptr;
  int dirmask = 0;                 // p_rgh = 0 box faces
  int batch_p = 4;
  struct {
    double inner_min = 2e-6;   // smallest FP32 inner relative tolerance
  } tune;
  // live timing of the pressure solve's fine-level operator kernel
  static constexpr int NEV = 256;
  bool timing = false;
  hipEvent_t ev[2 * NEV] = {};
  double t_sum_ms = 0.0;
  long long t_count = 0;
  double t_bytes = 0.0;
  // pinned host mirrors
  double* h_scal = nullptr;
  SolveStatus* h_status = nullptr;   // 4 slots
  ds_diagnostics diag_out{};
  double fuel_mass_prev = 0.0;
  int batch[3] = {8, 8, 8};
};

namespace {

int fail(ds_grid* g, int code, const char* fmt, ...) {
  if (g) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g->err = buf;
  }
  return code;
}

#define HIPCHK(g, call)                                                                  \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess) return fail(g, DS_ERR_HIP, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// Workspace layout: cell arrays, face arrays, then small scalar areas.
struct Layout {
  size_t off = 0;
  template <class T>
  T* take(char* base, size_t count) {
    T* ptr = base ? reinterpret_cast<T*>(base + off) : nullptr;
    off = align256(off + count * sizeof(T));
    return ptr;
  }
};

size_t carve(ds_grid* g, char* base) {
  Layout L;
  const long long n = g->n;
  g->alpha = L.take<double>(base, n);
  g->c = L.take<double>(base, n);
  g->omega = L.take<double>(base, n);
  g->T = L.take<double>(base, n);
  g->p = L.take<double>(base, n);
  g->u = L.take<double>(base, g->nu);
  g->v = L.take<double>(base, g->nv);
  g->w = L.take<double>(base, g->nw);
  g->a1 = L.take<double>(base, n);
  g->a_new = L.take<double>(base, n);
  g->c_new = L.take<double>(base, n);
  g->T_new = L.take<double>(base, n);
  g->om_new = L.take<double>(base, n);
  g->mraw = L.take<double>(base, n);
  g->mdot = L.take<double>(base, n);
  g->us = L.take<double>(base, g->nu);
  g->vs = L.take<double>(base, g->nv);
  g->ws = L.take<double>(base, g->nw);
  g->xi = L.take<double>(base, n);
  g->b = L.take<double>(base, n);
  g->r = L.take<double>(base, n);
  g->pd = L.take<double>(base, n);
  g->q = L.take<double>(base, n);
  g->diag = L.take<double>(base, n);
  g->qc = L.take<double>(base, n);
  g->adj = L.take<int>(base, n);
  g->partials = L.take<double>(base, (size_t)MAX_BLOCKS * MAX_RED);
  g->counters = L.take<unsigned>(base, CT_COUNT);
  g->scal = L.take<double>(base, SC_COUNT);
  g->status = L.take<SolveStatus>(base, 4);
  g->p_alt = L.take<double>(base, n);
  g->phi = L.take<double>(base, n);
  // FP64 multigrid levels (level 0 uses qc/diag of the pressure system)
  MgHier<double>& H = g->H64;
  H.lev[0].qc = g->qc;
  H.lev[0].diag = g->diag;
  for (int l = 0; l < H.nlev; ++l) {
    const long long nl = H.lev[l].n;
    if (l > 0) {
      H.lev[l].qc = L.take<double>(base, nl);
      H.lev[l].diag = L.take<double>(base, nl);
      H.r[l] = L.take<double>(base, nl);
    }
    H.x[l] = L.take<double>(base, nl);
    H.t[l] = L.take<double>(base, nl);
  }
  if (g->prm.precision == DS_PREC_MIXED) {
    MgHier<float>& F = g->H32;
    g->qc32 = L.take<float>(base, n);
    g->diag32 = L.take<float>(base, n);
    F.lev[0].qc = g->qc32;
    F.lev[0].diag = g->diag32;
    for (int l = 0; l < F.nlev; ++l) {
      const long long nl = F.lev[l].n;
      if (l > 0) {
        F.lev[l].qc = L.take<float>(base, nl);
        F.lev[l].diag = L.take<float>(base, nl);
        F.r[l] = L.take<float>(base, nl);
      }
      F.x[l] = L.take<float>(base, nl);
      F.t[l] = L.take<float>(base, nl);
    }
    g->e32 = L.take<float>(base, n);
    g->r32 = L.take<float>(base, n);
    g->p32 = L.take<float>(base, n);
    g->p32alt = L.take<float>(base, n);
    g->q32 = L.take<float>(base, n);
  }
  return L.off;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Multigrid shape: damped-Jacobi sweeps, coarsest-level sweeps and the
// smallest extent that is still coarsened (overridable for tuning through
// DSVOF_MG_NU, DSVOF_MG_COARSE, DSVOF_MG_MINDIM).
template <class T>
void build_hier(MgHier<T>& H, int nx, int ny, int nz, double h, double dt) {
  H.nlev = 0;
  double hl = h;
  int mindim = 8;
  if (const char* e = getenv("DSVOF_MG_NU")) H.nu = std::max(1, atoi(e));
  if (const char* e = getenv("DSVOF_MG_COARSE")) H.coarse_sweeps = std::max(2, atoi(e));
  if (const char* e = getenv("DSVOF_MG_MINDIM")) mindim = std::max(4, atoi(e));
  if (const char* e = getenv("DSVOF_MG_OMEGA")) H.omega = atof(e);
  for (;;) {
    Lev<T>& L = H.lev[H.nlev++];
    lev_dims(L, nx, ny, nz, dt / (hl * hl));
    if (std::min(nx, std::min(ny, nz)) < mindim || H.nlev == MG_MAXLEV) break;
    nx = (nx + 1) / 2;
    ny = (ny + 1) / 2;
    nz = (nz + 1) / 2;
    hl *= 2.0;
  }
}

int sync_status(ds_grid* g, int slot, hipStream_t s) {
  HIPCHK(g, hipMemcpyAsync(g->h_status + slot, g->status + slot, sizeof(SolveStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(g, hipStreamSynchronize(s));
  return DS_OK;
}

int init_status(ds_grid* g, int slot, double tol, int maxit, hipStream_t s) {
  SolveStatus init{};
  init.tol = tol;
  init.maxit = maxit;
  HIPCHK(g, hipMemcpyAsync(g->status + slot, &init, sizeof(init), hipMemcpyHostToDevice, s));
  return DS_OK;
}

// After a batch sync: add the durations of the operator launches that did
// work (the first `did` of the batch; later ones returned at once).
void accumulate_timing(ds_grid* g, int did, double bytes_per_launch) {
  for (int t = 0; t < did && t < ds_grid::NEV; ++t) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g->ev[2 * t], g->ev[2 * t + 1]) == hipSuccess) {
      g->t_sum_ms += ms;
      g->t_count += 1;
      g->t_bytes = bytes_per_launch;
    }
  }
}

// Iterations enqueued between host convergence tests: about half of the
// previous solve's count, so most solves finish in two or three batches.
int& batch_of(ds_grid* g, int sys) { return sys == 2 ? g->batch_p : g->batch[sys]; }

// FP64 preconditioned CG on the system in qc/diag (scale sc), right-hand side
// b, warm start in x.  sys: 0 = energy, 1 = species (Jacobi), 2 = pressure
// (multigrid when enabled, Jacobi otherwise).
int cg_solve64(ds_grid* g, int sys, double sc, double* x, hipStream_t s, int* iters, double* res, double tol) {
  int st;
  Lev<double> L = g->L0;
  L.sc = sc;
  L.qc = g->qc;
  L.diag = g->diag;
  MgHier<double>* H = nullptr;
  if (sys == 2 && g->prm.pressure_precond == 1) {
    H = &g->H64;
    H->lev[0] = L;
    mg_setup_levels(*H, g->dirmask, s);
  }
  SolveStatus* ss = g->status + sys;
  if ((st = init_status(g, sys, tol, g->prm.maxit, s)) != DS_OK) return st;
  launch_resid64(L, g->b, x, g->r, ss, g->partials, g->counters + CT_SOLVE0, true, s);
  launch_zero_if_flagged(x, g->n, ss, s);
  HIPCHK(g, hipGetLastError());
  if ((st = sync_status(g, sys, s)) != DS_OK) return st;
  if (!g->h_status[sys].done) {
    CgVecs<double> V{x, g->r, g->pd, g->p_alt, g->q};
    double* z = nullptr;
    cg_start(L, H, V, &z, ss, g->partials, g->counters + CT_SOLVE0, s);
    bool first = true;
    const bool timed = g->timing && H;
    while (!g->h_status[sys].done) {
      const int it0 = g->h_status[sys].it;
      const int m = timed ? std::min(batch_of(g, sys), (int)ds_grid::NEV) : batch_of(g, sys);
      for (int t = 0; t < m; ++t) {
        cg_iteration(L, H, V, &z, ss, g->partials, g->counters + CT_SOLVE0, first, s,
                     timed ? g->ev[2 * t] : nullptr, timed ? g->ev[2 * t + 1] : nullptr);
        first = false;
      }
      HIPCHK(g, hipGetLastError());
      if ((st = sync_status(g, sys, s)) != DS_OK) return st;
      if (timed) accumulate_timing(g, g->h_status[sys].it - it0, 48.0 * (double)g->n);
    }
  }
  const SolveStatus& h = g->h_status[sys];
  batch_of(g, sys) = std::max(2, std::min(256, h.it / 2 + 1));
  *iters = h.it;
  *res = h.res;
  if (sys == 2) g->diag_out.refinements_p = 0;
  return h.done == 1 ? DS_OK : DS_ERR_NOT_CONVERGED;
}

// Precision form of one solve: FP64 residual r = b - A x; FP32 preconditioned
// CG for the correction A e = r to an inner tolerance (FP32 vectors, operator
// and sweeps, FP64 dot products); x += e in FP64; repeat until ||r|| <= tol ||b||.
int cg_solve_mixed(ds_grid* g, int sys, double sc, double* x, hipStream_t s, int* iters, double* res, double tol) {
  int st;
  Lev<double> L = g->L0;
  L.sc = sc;
  L.qc = g->qc;
  L.diag = g->diag;
  Lev<float> F;
  lev_dims(F, L.nx, L.ny, L.nz, sc);
  F.qc = g->qc32;
  F.diag = g->diag32;
  launch_to_float(g->qc, g->qc32, g->n, s);
  launch_to_float(g->diag, g->diag32, g->n, s);
  MgHier<float>* H = nullptr;
  if (sys == 2 && g->prm.pressure_precond == 1) {
    H = &g->H32;
    H->lev[0] = F;
    mg_setup_levels(*H, g->dirmask, s);
  }
  SolveStatus* so = g->status + sys;
  SolveStatus* si = g->status + 3;
  const int max_rounds = 12;
  if ((st = init_status(g, sys, tol, g->prm.maxit, s)) != DS_OK) return st;
  launch_resid64(L, g->b, x, g->r, so, g->partials, g->counters + CT_SOLVE0, true, s);
  launch_zero_if_flagged(x, g->n, so, s);
  HIPCHK(g, hipGetLastError());
  if ((st = sync_status(g, sys, s)) != DS_OK) return st;
  int total = 0, rounds = 0, inner_fail = 0;
  while (!g->h_status[sys].done && rounds < max_rounds && !inner_fail) {
    // Ask the FP32 solve for the reduction still needed (with a margin), but
    // not below what FP32 arithmetic reliably attains.
    const double need = 0.5 * tol / std::max(g->h_status[sys].res, 1e-300);
    const double inner_tol = std::min(0.5, std::max(g->tune.inner_min, need));
    if ((st = init_status(g, 3, inner_tol, g->prm.maxit, s)) != DS_OK) return st;
    launch_inner_init<float>(F, g->r, g->r32, g->e32, si, g->partials, g->counters + CT_SOLVE1, s);
    g->h_status[3].it = 0;
    g->h_status[3].done = 0;
    CgVecs<float> V{g->e32, g->r32, g->p32, g->p32alt, g->q32};
    float* z = nullptr;
    cg_start(F, H, V, &z, si, g->partials, g->counters + CT_SOLVE0, s);
    bool first = true;
    const bool timed = g->timing && H;
    do {
      const int it0 = g->h_status[3].it;
      const int m = timed ? std::min(batch_of(g, sys), (int)ds_grid::NEV) : batch_of(g, sys);
      for (int t = 0; t < m; ++t) {
        cg_iteration(F, H, V, &z, si, g->partials, g->counters + CT_SOLVE0, first, s,
                     timed ? g->ev[2 * t] : nullptr, timed ? g->ev[2 * t + 1] : nullptr);
        first = false;
      }
      HIPCHK(g, hipGetLastError());
      if ((st = sync_status(g, 3, s)) != DS_OK) return st;
      if (timed) accumulate_timing(g, g->h_status[3].it - it0, 24.0 * (double)g->n);
    } while (!g->h_status[3].done);
    total += g->h_status[3].it;
    inner_fail = g->h_status[3].done == 2;
    launch_add_correction<float>(F, x, g->e32, s);
    launch_resid64(L, g->b, x, g->r, so, g->partials, g->counters + CT_SOLVE0, false, s);
    HIPCHK(g, hipGetLastError());
    if ((st = sync_status(g, sys, s)) != DS_OK) return st;
    ++rounds;
  }
  batch_of(g, sys) = std::max(2, std::min(256, total / std::max(1, 2 * rounds) + 1));
  *iters = total;
  *res = g->h_status[sys].res;
  if (sys == 2) g->diag_out.refinements_p = rounds;
  return g->h_status[sys].done == 1 ? DS_OK : DS_ERR_NOT_CONVERGED;
}

int solve(ds_grid* g, int sys, double sc, double* x, hipStream_t s, int* iters, double* res, double tol) {
  if (g->prm.precision == DS_PREC_MIXED) return cg_solve_mixed(g, sys, sc, x, s, iters, res, tol);
  return cg_solve64(g, sys, sc, x, s, iters, res, tol);
}
int solve(ds_grid* g, int sys, double sc, double* x, hipStream_t s, int* iters, double* res) {
  return solve(g, sys, sc, x, s, iters, res, g->prm.tol);
}

int solve_pressure_system(ds_grid* g, hipStream_t s, int* iters, double* res) {
  const DevParams& P = g->dp;
  return solve(g, 2, P.dt / (P.h * P.h), g->p, s, iters, res);
}

int evaporation_source(ds_grid* g, hipStream_t s) {
  const DevParams& P = g->dp;
  if (P.evaporation) {
    launch_interface(P, g->alpha, g->T, g->omega, g->u, g->v, g->w, g->mraw, g->adj, g->partials,
                     g->counters + CT_IFACE, g->scal, s);
  } else {
    launch_fill(g->mraw, 0.0, g->n, s);
    launch_fill(g->scal + SC_K, 0.0, 4, s);
  }
  launch_source(P, g->alpha, g->mraw, g->scal, g->mdot, g->a1, s);
  HIPCHK(g, hipGetLastError());
  return DS_OK;
}

int read_scalars(ds_grid* g, hipStream_t s) {
  HIPCHK(g, hipMemcpyAsync(g->h_scal, g->scal, SC_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(g, hipStreamSynchronize(s));
  return DS_OK;
}

int one_step(ds_grid* g, hipStream_t s) {
  const DevParams& P = g->dp;
  ds_diagnostics& D = g->diag_out;
  int rc = DS_OK, st;
  D.fuel_mass_before = g->fuel_mass_prev;
  // 1-2. evaporation source and liquid source
  if ((st = evaporation_source(g, s)) != DS_OK) return st;
  // 3. advection of alpha1 with the divergence-free part of u^n, c and T with u^n
  if (g->prm.liquid_transport) {
    launch_div_setup(P, g->u, g->v, g->w, g->qc, g->diag, g->b, s);
    st = solve(g, 2, P.dt / (P.h * P.h), g->phi, s, &D.iters_phi, &D.res_phi, g->prm.tol_phi);
    if (st == DS_ERR_NOT_CONVERGED) rc = st;
    else if (st != DS_OK) return st;
  } else {
    D.iters_phi = 0;
    D.res_phi = 0.0;
  }
  launch_advect(P, g->a1, g->omega, g->T, g->c, g->u, g->v, g->w, g->prm.liquid_transport ? g->phi : nullptr,
                g->a_new, g->c_new, g->T_new, g->partials, g->counters + CT_ADV, g->scal, s);
  // 5a. energy (warm start T')
  if (P.solve_energy) {
    launch_energy_setup(P, g->a_new, g->T_new, g->mdot, g->u, g->v, g->w, g->qc, g->diag, g->b, s);
    st = solve(g, 0, 1.0 / (P.h * P.h), g->T_new, s, &D.iters_T, &D.res_T);
    if (st == DS_ERR_NOT_CONVERGED) rc = st;
    else if (st != DS_OK) return st;
    std::swap(g->T, g->T_new);
  } else {
    D.iters_T = 0;
    D.res_T = 0.0;
  }
  // 5b. species (warm start omega' = c'/(rho_G theta))
  launch_species_setup(P, g->a_new, g->c_new, g->mdot, g->u, g->v, g->w, g->qc, g->diag, g->b, g->om_new, s);
  st = solve(g, 1, P.rho_G * P.D / (P.h * P.h), g->om_new, s, &D.iters_omega, &D.res_omega);
  if (st == DS_ERR_NOT_CONVERGED) rc = st;
  else if (st != DS_OK) return st;
  launch_species_update(P, g->a_new, g->c_new, g->mdot, g->om_new, g->u, g->v, g->w, g->c, g->omega,
                        g->partials, g->counters + CT_SPEC, g->scal, s);
  // 5c. momentum predictor with alpha'
  launch_predictor(P, g->a_new, g->xi, g->u, g->v, g->w, g->us, g->vs, g->ws, s);
  // 6. pressure (warm start p^n) and correction
  launch_pressure_setup(P, g->a_new, g->mdot, g->us, g->vs, g->ws, g->qc, g->diag, g->b, s);
  st = solve_pressure_system(g, s, &D.iters_p, &D.res_p);
  if (st == DS_ERR_NOT_CONVERGED) rc = st;
  else if (st != DS_OK) return st;
  launch_project(P, g->a_new, g->p, g->us, g->vs, g->ws, g->u, g->v, g->w, s);
  std::swap(g->alpha, g->a_new);
  // diagnostics
  launch_diagnostics(P, g->alpha, g->c, g->T, g->p, g->mdot, g->partials, g->counters + CT_DIAG, g->scal, s);
  HIPCHK(g, hipGetLastError());
  if ((st = read_scalars(g, s)) != DS_OK) return st;
  const double* sc = g->h_scal;
  D.K = sc[SC_K];
  D.n_interface = (int)sc[SC_NINT];
  D.B_L = sc[SC_BL];
  D.B_v = sc[SC_BV_ADV] + sc[SC_BV_DIFF];
  D.volume = sc[SC_VOL];
  D.fuel_mass = sc[SC_FUEL];
  D.mdot_total = sc[SC_MDOT];
  D.alpha_min = sc[SC_AMIN];
  D.alpha_max = sc[SC_AMAX];
  D.rho_G = P.rho_G;
  D.converged = rc == DS_OK;
  g->fuel_mass_prev = D.fuel_mass;
  if (sc[SC_NONFINITE] != 0.0) return fail(g, DS_ERR_NONFINITE, "non-finite values after the step");
  if (rc != DS_OK) fail(g, rc, "a linear solve reached maxit (T %d, omega %d, p %d iterations)", D.iters_T,
                        D.iters_omega, D.iters_p);
  return rc;
}

bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

}  // namespace

extern "C" {

int ds_create_grid(int nx, int ny, int nz, const ds_params* prm, ds_grid** out) {
  if (!out) return DS_ERR_ARG;
  *out = nullptr;
  if (!prm || nx < 2 || ny < 2 || nz < 2) return DS_ERR_ARG;
  const long long n = (long long)nx * ny * nz;
  if (n > (1LL << 31) - 1) return DS_ERR_ARG;
  if (!finite_pos(prm->h) || !finite_pos(prm->dt) || !finite_pos(prm->p) || !finite_pos(prm->T_amb) ||
      !finite_pos(prm->rho_L) || !finite_pos(prm->cp_L) || !finite_pos(prm->cp_G) || prm->k_L < 0 ||
      prm->k_G < 0 || !finite_pos(prm->D_v) || !finite_pos(prm->M_v) || !finite_pos(prm->M_G) ||
      !finite_pos(prm->T_ref) || !finite_pos(prm->p_ref) || !(prm->eps_int > 0 && prm->eps_int < 0.5) || !(prm->eps_gas >= prm->eps_int && prm->eps_gas <= 0.5) ||
      !finite_pos(prm->theta_min) || !(prm->tol > 0) || !(prm->tol_phi > 0) || prm->maxit < 1 || prm->s_max < 1 ||
      prm->eq_model < 0 || prm->eq_model > 1 || prm->bc_mode < 0 || prm->bc_mode > 2 ||
      prm->precision < 0 || prm->precision > 1 || !finite_pos(prm->r_fib) || prm->pressure_precond < 0 ||
      prm->pressure_precond > 1 || prm->liquid_transport < 0 || prm->liquid_transport > 1)
    return DS_ERR_ARG;
  if (prm->eq_model == DS_EQ_PENG_ROBINSON &&
      (!finite_pos(prm->Tc) || !finite_pos(prm->Pc) || !finite_pos(prm->Tc_G) || !finite_pos(prm->Pc_G)))
    return DS_ERR_ARG;
  ds_grid* g = new ds_grid();
  g->prm = *prm;
  g->n = n;
  g->nu = (long long)(nx + 1) * ny * nz;
  g->nv = (long long)nx * (ny + 1) * nz;
  g->nw = (long long)nx * ny * (nz + 1);
  DevParams& P = g->dp;
  P.nx = nx;
  P.ny = ny;
  P.nz = nz;
  P.n = n;
  P.smax = prm->s_max;
  P.h = prm->h;
  P.dt = prm->dt;
  P.p = prm->p;
  P.T_amb = prm->T_amb;
  P.rho_L = prm->rho_L;
  P.cp_L = prm->cp_L;
  P.k_L = prm->k_L;
  P.cp_G = prm->cp_G;
  P.k_G = prm->k_G;
  P.D = prm->D_v;
  P.dh = prm->dh_ev;
  P.M_v = prm->M_v;
  P.M_G = prm->M_G;
  for (int a = 0; a < 3; ++a) {
    P.g[a] = prm->g[a];
    P.x0[a] = prm->x0[a];
  }
  P.xi0 = prm->xi0;
  P.Df = prm->Df;
  P.r_fib = prm->r_fib;
  P.w_in = prm->w_in;
  P.Tc = prm->Tc;
  P.Pc = prm->Pc;
  P.om = prm->acentric;
  P.Tc_G = prm->Tc_G;
  P.Pc_G = prm->Pc_G;
  P.om_G = prm->acentric_G;
  P.kij = prm->kij;
  P.T_ref = prm->T_ref;
  P.p_ref = prm->p_ref;
  P.eps = prm->eps_int;
  P.eps_gas = prm->eps_gas;
  P.theta_min = prm->theta_min;
  P.eq_model = prm->eq_model;
  P.solve_energy = prm->solve_energy;
  P.evaporation = prm->evaporation;
  // gas density, eq. 24, for the ambient gas at (T_amb, p)
  const double Z = prm->eq_model == DS_EQ_PENG_ROBINSON
                       ? host_pr_Z(prm->T_amb, prm->p, prm->Tc_G, prm->Pc_G, prm->acentric_G)
                       : 1.0;
  P.rho_G = prm->p * prm->M_G / (Z * R_GAS * prm->T_amb);
  // box faces: x/y walls, z- inlet (open in natural convection), z+ outlet
  for (int ax = 0; ax < 3; ++ax)
    for (int sd = 0; sd < 2; ++sd) {
      int kind;
      if (prm->bc_mode == DS_BC_FARFIELD) kind = FARFIELD;
      else if (ax < 2) kind = WALL;
      else if (sd == 1) kind = OPEN;
      else kind = prm->bc_mode == DS_BC_FORCED ? INLET : OPEN;
      P.kind[ax * 2 + sd] = kind;
    }
  for (int ax = 0; ax < 3; ++ax)
    for (int sd = 0; sd < 2; ++sd)
      if (pressure_dirichlet(P.kind[ax * 2 + sd])) g->dirmask |= 1 << (ax * 2 + sd);
  lev_dims(g->L0, nx, ny, nz, 1.0);
  if (const char* e = getenv("DSVOF_INNER_MIN")) g->tune.inner_min = atof(e);
  if (prm->pressure_precond == 1) build_hier(g->H64, nx, ny, nz, prm->h, prm->dt);
  if (prm->precision == DS_PREC_MIXED) {
    if (prm->pressure_precond == 1) build_hier(g->H32, nx, ny, nz, prm->h, prm->dt);
    else lev_dims(g->H32.lev[0], nx, ny, nz, 1.0), g->H32.nlev = 1;
  }
  g->ws_bytes = carve(g, nullptr);
  if (hipHostMalloc((void**)&g->h_scal, SC_COUNT * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&g->h_status, 4 * sizeof(SolveStatus), hipHostMallocDefault) != hipSuccess) {
    if (g->h_scal) (void)hipHostFree(g->h_scal);
    delete g;
    return DS_ERR_HIP;
  }
  *out = g;
  return DS_OK;
}

int ds_destroy_grid(ds_grid* g) {
  if (!g) return DS_ERR_ARG;
  for (int e = 0; e < 2 * ds_grid::NEV; ++e)
    if (g->ev[e]) (void)hipEventDestroy(g->ev[e]);
  if (g->h_scal) (void)hipHostFree(g->h_scal);
  if (g->h_status) (void)hipHostFree(g->h_status);
  delete g;
  return DS_OK;
}

size_t ds_workspace_bytes(const ds_grid* g) { return g ? g->ws_bytes : 0; }

int ds_set_fields(ds_grid* g, const double* alpha, const double* T, const double* omega, const double* u,
                  const double* v, const double* w, const double* p, void* workspace, size_t workspace_bytes,
                  void* stream) {
  if (!g) return DS_ERR_ARG;
  if (!alpha || !T || !omega || !u || !v || !w || !p || !workspace)
    return fail(g, DS_ERR_ARG, "null pointer argument");
  if (workspace_bytes < g->ws_bytes)
    return fail(g, DS_ERR_ARG, "workspace too small: %zu < %zu bytes", workspace_bytes, g->ws_bytes);
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(g, DS_ERR_ARG, "workspace not 256-byte aligned");
  hipStream_t s = S(stream);
  carve(g, static_cast<char*>(workspace));
  const size_t nb = g->n * sizeof(double);
  HIPCHK(g, hipMemcpyAsync(g->alpha, alpha, nb, hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(g->T, T, nb, hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(g->omega, omega, nb, hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(g->p, p, nb, hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(g->u, u, g->nu * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(g->v, v, g->nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(g->w, w, g->nw * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemsetAsync(g->counters, 0, CT_COUNT * sizeof(unsigned), s));
  HIPCHK(g, hipMemsetAsync(g->scal, 0, SC_COUNT * sizeof(double), s));
  HIPCHK(g, hipMemsetAsync(g->mdot, 0, nb, s));
  HIPCHK(g, hipMemsetAsync(g->mraw, 0, nb, s));
  HIPCHK(g, hipMemsetAsync(g->phi, 0, nb, s));
  launch_xi(g->dp, g->xi, s);
  // conservative vapour variable c = rho_G theta omega (gas fraction only)
  launch_c_from_omega(g->dp, g->alpha, g->omega, g->c, s);
  HIPCHK(g, hipGetLastError());
  g->bound = true;
  int st;
  launch_diagnostics(g->dp, g->alpha, g->c, g->T, g->p, g->mdot, g->partials, g->counters + CT_DIAG, g->scal, s);
  HIPCHK(g, hipGetLastError());
  if ((st = read_scalars(g, s)) != DS_OK) return st;
  g->fuel_mass_prev = g->h_scal[SC_FUEL];
  if (g->h_scal[SC_NONFINITE] != 0.0) return fail(g, DS_ERR_NONFINITE, "non-finite input fields");
  g->err.clear();
  return DS_OK;
}

int ds_get_fields(ds_grid* g, double* alpha, double* T, double* omega, double* u, double* v, double* w,
                  double* p, void* stream) {
  if (!g) return DS_ERR_ARG;
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  hipStream_t s = S(stream);
  const size_t nb = g->n * sizeof(double);
  if (alpha) HIPCHK(g, hipMemcpyAsync(alpha, g->alpha, nb, hipMemcpyDeviceToDevice, s));
  if (T) HIPCHK(g, hipMemcpyAsync(T, g->T, nb, hipMemcpyDeviceToDevice, s));
  if (omega) HIPCHK(g, hipMemcpyAsync(omega, g->omega, nb, hipMemcpyDeviceToDevice, s));
  if (p) HIPCHK(g, hipMemcpyAsync(p, g->p, nb, hipMemcpyDeviceToDevice, s));
  if (u) HIPCHK(g, hipMemcpyAsync(u, g->u, g->nu * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (v) HIPCHK(g, hipMemcpyAsync(v, g->v, g->nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (w) HIPCHK(g, hipMemcpyAsync(w, g->w, g->nw * sizeof(double), hipMemcpyDeviceToDevice, s));
  return DS_OK;
}

int ds_step(ds_grid* g, int nsteps, void* stream) {
  if (!g || nsteps < 0) return DS_ERR_ARG;
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  int rc = DS_OK;
  for (int n = 0; n < nsteps; ++n) {
    int st = one_step(g, S(stream));
    if (st == DS_ERR_NOT_CONVERGED) rc = st;
    else if (st != DS_OK) return st;
  }
  if (rc == DS_OK) g->err.clear();
  return rc;
}


int ds_solve_pressure(ds_grid* g, void* stream, int* iters, double* rel_res) {
  if (!g) return DS_ERR_ARG;
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  hipStream_t s = S(stream);
  const DevParams& P = g->dp;
  int st;
  if ((st = evaporation_source(g, s)) != DS_OK) return st;
  launch_predictor(P, g->alpha, g->xi, g->u, g->v, g->w, g->us, g->vs, g->ws, s);
  launch_pressure_setup(P, g->alpha, g->mdot, g->us, g->vs, g->ws, g->qc, g->diag, g->b, s);
  int it = 0;
  double res = 0.0;
  st = solve_pressure_system(g, s, &it, &res);
  if (st != DS_OK && st != DS_ERR_NOT_CONVERGED) return st;
  launch_project(P, g->alpha, g->p, g->us, g->vs, g->ws, g->u, g->v, g->w, s);
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipStreamSynchronize(s));
  g->diag_out.iters_p = it;
  g->diag_out.res_p = res;
  if (iters) *iters = it;
  if (rel_res) *rel_res = res;
  return st;
}

int ds_evaporation_rate(ds_grid* g, double* kg_per_s, double* mdot_or_null, void* stream) {
  if (!g) return DS_ERR_ARG;
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  hipStream_t s = S(stream);
  int st;
  if ((st = evaporation_source(g, s)) != DS_OK) return st;
  launch_diagnostics(g->dp, g->alpha, g->c, g->T, g->p, g->mdot, g->partials, g->counters + CT_DIAG, g->scal, s);
  if (mdot_or_null) HIPCHK(g, hipMemcpyAsync(mdot_or_null, g->mdot, g->n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipGetLastError());
  if ((st = read_scalars(g, s)) != DS_OK) return st;
  g->diag_out.K = g->h_scal[SC_K];
  g->diag_out.mdot_total = g->h_scal[SC_MDOT];
  g->diag_out.n_interface = (int)g->h_scal[SC_NINT];
  if (kg_per_s) *kg_per_s = g->h_scal[SC_MDOT];
  return DS_OK;
}

int ds_droplet_volume(ds_grid* g, double* m3, void* stream) {
  if (!g || !m3) return DS_ERR_ARG;
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  hipStream_t s = S(stream);
  launch_diagnostics(g->dp, g->alpha, g->c, g->T, g->p, g->mdot, g->partials, g->counters + CT_DIAG, g->scal, s);
  HIPCHK(g, hipGetLastError());
  int st;
  if ((st = read_scalars(g, s)) != DS_OK) return st;
  *m3 = g->h_scal[SC_VOL];
  return DS_OK;
}

int ds_get_internal(ds_grid* g, int which, double* dst, size_t count, void* stream) {
  if (!g || !dst) return DS_ERR_ARG;
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  hipStream_t s = S(stream);
  const double* src = nullptr;
  size_t n = (size_t)g->n;
  switch (which) {
    case DS_FIELD_MDOT_RAW: src = g->mraw; break;
    case DS_FIELD_MDOT: src = g->mdot; break;
    case DS_FIELD_ALPHA1: src = g->a1; break;
    case DS_FIELD_C: src = g->c; break;
    case DS_FIELD_USTAR: src = g->us; n = (size_t)g->nu; break;
    case DS_FIELD_VSTAR: src = g->vs; n = (size_t)g->nv; break;
    case DS_FIELD_WSTAR: src = g->ws; n = (size_t)g->nw; break;
    case DS_FIELD_ADJ: break;
    default: return fail(g, DS_ERR_ARG, "unknown internal field %d", which);
  }
  if (count != n) return fail(g, DS_ERR_ARG, "buffer holds %zu values, field has %zu", count, n);
  if (which == DS_FIELD_ADJ) launch_int_to_double(g->adj, dst, g->n, s);
  else HIPCHK(g, hipMemcpyAsync(dst, src, n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipGetLastError());
  return DS_OK;
}

int ds_set_kernel_timing(ds_grid* g, int enable) {
  if (!g) return DS_ERR_ARG;
  if (enable && !g->ev[0])
    for (int e = 0; e < 2 * ds_grid::NEV; ++e) HIPCHK(g, hipEventCreate(&g->ev[e]));
  g->timing = enable != 0;
  g->t_sum_ms = 0.0;
  g->t_count = 0;
  return DS_OK;
}

int ds_get_kernel_timing(const ds_grid* g, double* avg_us, long long* launches, double* bytes_per_launch) {
  if (!g) return DS_ERR_ARG;
  if (avg_us) *avg_us = g->t_count ? 1e3 * g->t_sum_ms / (double)g->t_count : 0.0;
  if (launches) *launches = g->t_count;
  if (bytes_per_launch) *bytes_per_launch = g->t_bytes;
  return DS_OK;
}

int ds_time_operator_kernel(ds_grid* g, int reps, double* avg_us, double* bytes_per_launch, void* stream) {
  if (!g || reps < 1 || !avg_us) return DS_ERR_ARG;
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  hipStream_t s = S(stream);
  if (!g->ev[0])
    for (int e = 0; e < 2 * ds_grid::NEV; ++e) HIPCHK(g, hipEventCreate(&g->ev[e]));
  SolveStatus init{};
  init.beta = 0.5;
  init.rz = 1.0;
  init.tol = 0.0;
  init.maxit = 1 << 30;
  SolveStatus* st = g->status + 3;
  HIPCHK(g, hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, s));
  double us;
  const DevParams& P = g->dp;
  if (g->prm.precision == DS_PREC_MIXED) {
    Lev<float> F;
    lev_dims(F, P.nx, P.ny, P.nz, P.dt / (P.h * P.h));
    F.qc = g->qc32;
    F.diag = g->diag32;
    us = replay_operator_kernel<float>(F, g->r32, g->p32, g->p32alt, g->q32, st, g->partials,
                                       g->counters + CT_MISC, reps, s, g->ev[0], g->ev[1]);
    if (bytes_per_launch) *bytes_per_launch = 24.0 * (double)g->n;
  } else {
    Lev<double> L = g->L0;
    L.sc = P.dt / (P.h * P.h);
    L.qc = g->qc;
    L.diag = g->diag;
    us = replay_operator_kernel<double>(L, g->r, g->pd, g->p_alt, g->q, st, g->partials, g->counters + CT_MISC,
                                        reps, s, g->ev[0], g->ev[1]);
    if (bytes_per_launch) *bytes_per_launch = 48.0 * (double)g->n;
  }
  if (us < 0) return fail(g, DS_ERR_HIP, "event timing failed");
  *avg_us = us;
  return DS_OK;
}

int ds_get_diagnostics(const ds_grid* g, ds_diagnostics* out) {
  if (!g || !out) return DS_ERR_ARG;
  *out = g->diag_out;
  return DS_OK;
}

const char* ds_last_error(const ds_grid* g) { return g ? g->err.c_str() : "null handle"; }

}  // extern "C"
