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

const char* dsv_noalloc_last_error();   // noalloc.hip: the thread's last handle-free error

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
    if (std::fabs(dz) <= 4.5e-16 * std::fabs(z)) break;
  }
  return z;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Arrays of the FP32-multigrid pressure solve: its operator (FP64 and the
// setup's FP32 copies), right-hand side, residuals, directions, A p and the
// reduction scratch of its kernels.
struct PBufs {
  double *qc = nullptr, *diag = nullptr, *b = nullptr, *r = nullptr, *q = nullptr;
  double *pd = nullptr, *p_alt = nullptr;   // FP64 directions (the FP64 form)
  float *qc32 = nullptr, *diag32 = nullptr, *r32 = nullptr, *p32 = nullptr, *p32alt = nullptr;
  double* partials = nullptr;
  unsigned* counters = nullptr;
};

}  // namespace

struct ds_grid {
  ds_params prm{};
  DevParams dp{};
  LaunchShape shape{};             // launch shapes of this handle's solver kernels
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
  int* band = nullptr;             // per-block lists of interface cells
  int* band_count = nullptr;
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
  double* zj = nullptr;            // Jacobi z = r/diag (FP64 solves)
  float* zj32 = nullptr;           // the same for the FP32 rounds
  double* r_alt = nullptr;         // second residual buffer of the Neumann-preconditioned solves
  ViscVecs visc{};                 // implicit viscous solve (viscous = 1): vectors over the faces [u | v | w]
  // variable-density gas (gas_density = 1): the state's rho_G, the advected state's rho_G', eq. 7's
  // compressibility term and the vapour mass per gas volume rho_G omega the advection carries
  double *rg = nullptr, *rg_p = nullptr, *scomp = nullptr, *qv = nullptr;
  // geometric advection (advection = 1): the planes of the surface cells (n_x, n_y, n_z, s; written only where
  // tol < alpha1 < 1 - tol) and the liquid fluxes per face
  double* geo_pl[4] = {};
  double* geo_F[3] = {};
  int batch_visc = 4;
  float* r32alt = nullptr;
  int dirmask = 0;                 // p_rgh = 0 box faces
  int batch_p[2] = {4, 4};         // pressure, then any other pressure-type system (phi, adjoints)
  int f32_sys = -1;                // system whose FP32 copies (qc32, diag32) the last setup wrote
  // The liquid-transport potential's operator (face coefficient 1/dt everywhere, the pressure's box faces)
  // does not change between steps: in the precision form's multigrid path it has its own FP64 q and FP32
  // hierarchy q and diag (H32phi, whose r, x, t scratch is H32's), built by its first solve.
  double* phi_qc = nullptr;
  float* phi_q[MG_MAXLEV] = {};
  float* phi_d[MG_MAXLEV] = {};
  MgHier<float> H32phi;
  bool phi_ready = false;          // phi_qc, phi_q, phi_d and H32phi hold the operator
  bool phi_op = false;             // the solve in progress is the potential's, on those arrays
  struct {
    double inner_min = 1e-3;   // smallest FP32 inner relative tolerance per round (pressure-type)
    double inner_min_jac = 1e-6;  // the same for the energy and species systems
    int mg32 = 1;                 // multigrid systems: FP64 CG with the FP32 V-cycle
    int neumann = 1;              // energy and species: Neumann-polynomial preconditioner (vectorised grids)
    int round_test = 1;           // energy and species FP32 rounds: one host test per round (0: also test the inner solve)
    int const_q = 1;              // potential's fine level: the coloured sweep takes its constant q from a register
    int graphs = 1;               // replay pairs of multigrid-CG iterations as HIP graphs
    int phi_direct = 1;           // the liquid-transport potential by the direct (diagonalised) solve
    int extrap = 1;               // species warm start plus the previous step's solve correction
    int overlap = 1;              // predictor and pressure on a second stream, concurrent with energy and species
  } tune;
  // the species solve's correction of its warm start in the last ds_step (omega~ - omega'); valid while
  // corr_ok (cleared by ds_set_fields; recording and the adjoint's replays neither read nor write it)
  double* om_corr = nullptr;
  bool corr_ok = false;
  bool recording = false;
  // The pressure solve's arrays: pb[0] the ones shared with the other solves; pb[1] its own set, carved
  // where ds_step runs the predictor and the pressure on a second stream (s2) while the energy and species
  // solves run on the caller's (precision form with the FP32 V-cycle, ambient gas, inviscid step)
  PBufs pb[2];
  bool pb_own = false;
  bool s2_failed = false;   // the second stream or its events could not be created: one stream
  hipStream_t s2 = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool fdm_ok = false;             // the grid's potential system takes the direct solve
  // Graphs of two FP32-multigrid CG iterations, keyed by what their launches
  // hold: solution and direction buffers, V-cycle output, system scale.  The
  // capture stream is the handle's own (default priority); replays go to the
  // caller's stream.
  struct Mg32Graph {
    hipGraphExec_t ex = nullptr;
    const void* x = nullptr;
    const void* p = nullptr;
    const void* z = nullptr;
    double sc = 0.0;
  };
  static constexpr int NGRAPH = 8;
  Mg32Graph graphs[NGRAPH];
  int graph_next = 0;
  hipStream_t cap_stream = nullptr;
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
  // FP32 rounds of the precision form: inner iterations the previous solve of
  // each system took in its first, second, third (and later) round; the first
  // round needs more than the later ones
  int batch_round[3][3] = {{8, 8, 8}, {8, 8, 8}, {8, 8, 8}};
  // differentiation form: arrays carved from the caller's tape
  char* tape = nullptr;
  size_t tape_bytes = 0, tape_slot_off = 0;
  int tape_steps = 0, tape_ckpt = 0;
  bool recorded = false;
  double fuel_mass_final = 0.0;
  ds_diagnostics diag_final{};
  double *A_al = nullptr, *A_c = nullptr, *A_om = nullptr, *A_T = nullptr, *A_ab = nullptr, *A_md = nullptr;
  double *A_cp = nullptr, *A_Tp = nullptr, *A_a1 = nullptr, *lam = nullptr, *grad = nullptr;
  double *A_U[3] = {}, *A_Us[3] = {}, *A_Ul[3] = {}, *Q[6] = {};
  double* h_grad = nullptr;          // pinned host mirror of grad
  IfaceRecords irec{};               // records of the adjoint interface stage (tape arrays)
  int adj_iters[4] = {0, 0, 0, 0};   // adjoint solve iterations: p, omega, T, phi (last ds_adjoint)
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

// Graphs hold workspace addresses: dropped whenever the workspace is bound.
void drop_graphs(ds_grid* g) {
  for (auto& e : g->graphs) {
    if (e.ex) (void)hipGraphExecDestroy(e.ex);
    e = ds_grid::Mg32Graph{};
  }
}

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
  g->om_corr = L.take<double>(base, n);
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
  g->band = L.take<int>(base, (size_t)interface_band_capacity(n));
  g->band_count = L.take<int>(base, 2 * MAX_BLOCKS + 1);   // counts, then offsets
  g->partials = L.take<double>(base, (size_t)MAX_BLOCKS * MAX_RED);
  g->counters = L.take<unsigned>(base, CT_COUNT);
  g->scal = L.take<double>(base, SC_COUNT);
  g->status = L.take<SolveStatus>(base, 4);
  g->p_alt = L.take<double>(base, n);
  g->phi = L.take<double>(base, n);
  g->zj = L.take<double>(base, n);
  g->r_alt = L.take<double>(base, n);
  if (g->prm.gas_density) {
    g->rg = L.take<double>(base, n);
    g->rg_p = L.take<double>(base, n);
    g->scomp = L.take<double>(base, n);
    g->qv = L.take<double>(base, n);
  }
  g->dp.rg = g->rg;   // stages read the state's gas density unless they set their own
  if (g->prm.advection) {
    for (int q = 0; q < 4; ++q) g->geo_pl[q] = L.take<double>(base, n);
    g->geo_F[0] = L.take<double>(base, g->nu);
    g->geo_F[1] = L.take<double>(base, g->nv);
    g->geo_F[2] = L.take<double>(base, g->nw);
  }
  if (g->prm.viscous) {
    const long long nf = visc_faces(g->dp);
    double** vv[6] = {&g->visc.x, &g->visc.b, &g->visc.d, &g->visc.r, &g->visc.p, &g->visc.q};
    for (double** v : vv) *v = L.take<double>(base, nf);
  }
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
    g->zj32 = L.take<float>(base, n);
    g->r32alt = L.take<float>(base, n);
    g->phi_qc = L.take<double>(base, n);
    for (int l = 0; l < F.nlev; ++l) {
      g->phi_q[l] = L.take<float>(base, F.lev[l].n);
      g->phi_d[l] = L.take<float>(base, F.lev[l].n);
    }
  }
  g->phi_ready = false;
  g->pb[0] = PBufs{g->qc,   g->diag,   g->b,   g->r,      g->q,        g->pd,       g->p_alt,
                   g->qc32, g->diag32, g->r32, g->p32, g->p32alt, g->partials, g->counters};
  if (g->pb_own) {
    PBufs& B = g->pb[1];
    B = PBufs{};
    B.qc = L.take<double>(base, n);
    B.diag = L.take<double>(base, n);
    B.b = L.take<double>(base, n);
    B.r = L.take<double>(base, n);
    B.q = L.take<double>(base, n);
    if (g->prm.precision == DS_PREC_MIXED) {
      B.qc32 = L.take<float>(base, n);
      B.diag32 = L.take<float>(base, n);
      B.r32 = L.take<float>(base, n);
      B.p32 = L.take<float>(base, n);
      B.p32alt = L.take<float>(base, n);
    } else {
      B.pd = L.take<double>(base, n);
      B.p_alt = L.take<double>(base, n);
    }
    B.partials = L.take<double>(base, (size_t)MAX_BLOCKS * MAX_RED);
    B.counters = L.take<unsigned>(base, CT_COUNT);
  } else {
    g->pb[1] = PBufs{};
  }
  return L.off;
}

// State of one step boundary on the tape: the state at the start of step k,
// and the solver outputs of step k-1 that the reverse sweep reuses (the
// liquid-transport potential, which is also step k's warm start, and the
// species solution omega~).
struct Slot {
  double *alpha, *c, *omega, *T, *p, *phi, *omt, *u, *v, *w;
};

size_t slot_bytes(const ds_grid* g) {
  return 7 * align256(g->n * sizeof(double)) + align256(g->nu * sizeof(double)) +
         align256(g->nv * sizeof(double)) + align256(g->nw * sizeof(double));
}

int tape_nckpt(int nsteps, int ckpt) { return (nsteps + ckpt - 1) / ckpt; }
int tape_nslots(int nsteps, int ckpt) { return tape_nckpt(nsteps, ckpt) + 1 + (ckpt > 1 ? ckpt - 1 : 0); }

// Bytes of the adjoint arrays and accumulators at the head of the tape (the
// layout carve_tape produces).
size_t tape_adjoint_bytes(const ds_grid* g) {
  const size_t cb = align256(g->n * sizeof(double));
  const size_t fb = align256(g->nu * sizeof(double)) + align256(g->nv * sizeof(double)) +
                    align256(g->nw * sizeof(double));
  // 10 adjoint cell arrays and 11 of interface records, the records' list of cells, 5 face arrays per axis
  return 21 * cb + align256(g->n * sizeof(int)) + 5 * fb + align256(GR_COUNT * sizeof(double)) +
         align256(2 * sizeof(unsigned));
}

size_t tape_total_bytes(const ds_grid* g, int nsteps, int ckpt) {
  return tape_adjoint_bytes(g) + (size_t)tape_nslots(nsteps, ckpt) * slot_bytes(g);
}

// Tape layout: adjoint arrays, gradient accumulators, then the slots
// (checkpoints at steps 0, C, 2C, ..., the final state, and C-1 segment slots).
void carve_tape(ds_grid* g, char* base) {
  Layout L;
  const long long n = g->n;
  const long long nf[3] = {g->nu, g->nv, g->nw};
  g->A_al = L.take<double>(base, n);
  g->A_c = L.take<double>(base, n);
  g->A_om = L.take<double>(base, n);
  g->A_T = L.take<double>(base, n);
  g->A_ab = L.take<double>(base, n);
  g->A_md = L.take<double>(base, n);
  g->A_cp = L.take<double>(base, n);
  g->A_Tp = L.take<double>(base, n);
  g->A_a1 = L.take<double>(base, n);
  g->lam = L.take<double>(base, n);
  for (int a = 0; a < 3; ++a) {
    g->A_U[a] = L.take<double>(base, nf[a]);
    g->A_Us[a] = L.take<double>(base, nf[a]);
    g->A_Ul[a] = L.take<double>(base, nf[a]);
    g->Q[2 * a] = L.take<double>(base, nf[a]);
    g->Q[2 * a + 1] = L.take<double>(base, nf[a]);
  }
  g->grad = L.take<double>(base, GR_COUNT);
  // the interface stage's records (gathered per target in a fixed order)
  IfaceRecords& R = g->irec;
  for (int q = 0; q < 3; ++q) R.gb[q] = L.take<double>(base, n);
  R.om = L.take<double>(base, n);
  for (int q = 0; q < 3; ++q) R.f[q] = L.take<double>(base, n);
  for (int q = 0; q < 3; ++q) R.gsf[q] = L.take<double>(base, n);
  R.hit = L.take<double>(base, n);
  R.list = L.take<int>(base, n);
  R.rmax = L.take<unsigned>(base, 2);
  R.nlist = R.rmax + 1;
  g->tape_slot_off = L.off;
}

// Recording and the adjoint's replays run steps without the species
// warm-start correction (which moves a solve within its tolerance); none is
// valid afterwards.  (The second stream stays: it changes no result.)
struct RecordingScope {
  ds_grid* g;
  explicit RecordingScope(ds_grid* g_) : g(g_) {
    g->recording = true;
    g->corr_ok = false;
  }
  ~RecordingScope() {
    g->recording = false;
    g->corr_ok = false;
  }
};

Slot slot_at(const ds_grid* g, int idx) {
  char* p = g->tape + g->tape_slot_off + (size_t)idx * slot_bytes(g);
  Slot sl;
  const size_t cb = align256(g->n * sizeof(double));
  double** cells[7] = {&sl.alpha, &sl.c, &sl.omega, &sl.T, &sl.p, &sl.phi, &sl.omt};
  for (int q = 0; q < 7; ++q) {
    *cells[q] = reinterpret_cast<double*>(p);
    p += cb;
  }
  sl.u = reinterpret_cast<double*>(p);
  p += align256(g->nu * sizeof(double));
  sl.v = reinterpret_cast<double*>(p);
  p += align256(g->nv * sizeof(double));
  sl.w = reinterpret_cast<double*>(p);
  return sl;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Multigrid shape: damped-Jacobi sweeps, coarsest-level sweeps and the
// smallest extent that is still coarsened (overridable for tuning through
// DSVOF_MG_NU, DSVOF_MG_COARSE, DSVOF_MG_MINDIM, DSVOF_MG_TAIL).
template <class T>
void build_hier(MgHier<T>& H, int nx, int ny, int nz, double h, double dt) {
  H.nlev = 0;
  double hl = h;
  int mindim = 8;
  if (const char* e = getenv("DSVOF_MG_NU")) H.nu = H.nu_fine = std::max(1, atoi(e));
  if (const char* e = getenv("DSVOF_MG_NU_FINE")) H.nu_fine = std::max(1, atoi(e));
  if (const char* e = getenv("DSVOF_MG_COARSE")) H.coarse_sweeps = std::max(2, atoi(e));
  if (const char* e = getenv("DSVOF_MG_MINDIM")) mindim = std::max(4, atoi(e));
  if (const char* e = getenv("DSVOF_MG_OMEGA")) H.omega = atof(e);
  if (const char* e = getenv("DSVOF_MG_TAIL")) H.tail = atoi(e);
  if (const char* e = getenv("DSVOF_MG_RB")) H.rb = atoi(e);
  if (const char* e = getenv("DSVOF_MG_RB_NU")) H.nu_rb = std::max(1, atoi(e));
  if (const char* e = getenv("DSVOF_MG_RB_W")) H.w_rb = atof(e);
  if (const char* e = getenv("DSVOF_MG_RB_MINPLANES")) H.rb_min_planes = std::max(1, atoi(e));
  if (const char* e = getenv("DSVOF_MG_RB_THREADS")) H.rb_threads = std::max(0LL, atoll(e));
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

// Both status slots a and b to the host with one synchronisation.
int sync_status2(ds_grid* g, int a, int b, hipStream_t s) {
  HIPCHK(g, hipMemcpyAsync(g->h_status + a, g->status + a, sizeof(SolveStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(g, hipMemcpyAsync(g->h_status + b, g->status + b, sizeof(SolveStatus), hipMemcpyDeviceToHost, s));
  HIPCHK(g, hipStreamSynchronize(s));
  return DS_OK;
}

int init_status(ds_grid* g, int slot, double tol, int maxit, hipStream_t s) {
  launch_init_status(g->status + slot, tol, maxit, s);
  HIPCHK(g, hipGetLastError());
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

// Iterations enqueued before the first host convergence test: the previous
// count of the same system (it barely changes from step to step), then a
// quarter of it per test; so most solves take one test and enqueue few
// iterations past convergence (each of those still costs its launches).
int& batch_of(ds_grid* g, int sys, const double* x) {
  return sys == 2 ? g->batch_p[x == g->p ? 0 : 1] : g->batch[sys];
}
int batch_size(int expected, bool first) { return first ? std::max(2, expected) : std::max(2, expected / 4); }

// The precision form's FP32 copies of the operator, written by the setup of
// system sys next to the FP64 arrays; the following solve of that system then
// skips its conversion passes.
F32Out f32_out(ds_grid* g, int sys) {
  F32Out fo;
  if (g->prm.precision != DS_PREC_MIXED) return fo;
  fo.q = g->qc32;
  fo.d = g->diag32;
  fo.mg = sys == 2 && g->prm.pressure_precond == 1;
  fo.sc = (double)(float)(g->dp.dt / (g->dp.h * g->dp.h));   // scale of the FP32 fine level (sys 2)
  g->f32_sys = sys;
  return fo;
}
// The pressure setup's FP32 copies into the pressure's own arrays (pb[1]).
F32Out f32_out_own(ds_grid* g) {
  F32Out fo;
  fo.q = g->pb[1].qc32;
  fo.d = g->pb[1].diag32;
  fo.mg = true;
  fo.sc = (double)(float)(g->dp.dt / (g->dp.h * g->dp.h));
  return fo;
}
bool take_f32(ds_grid* g, int sys) {
  const bool ready = g->f32_sys == sys;
  g->f32_sys = -1;
  return ready;
}

// Pressure-type systems (pressure, liquid-transport potential): the marching
// kernels form the diagonal from q and the p = 0 faces instead of loading it.
// For the pressure the result equals the setup's stored diagonal bit for bit
// (same terms, same order); for the potential it differs by at most an ulp.
void pressure_type(const ds_grid* g, int sys, Lev<double>& L) {
  if (sys != 2) return;
  L.dfly = 1;
  L.dmask = g->dirmask;
}

// FP64 preconditioned CG on the system in qc/diag (scale sc), right-hand side
// b, warm start in x.  sys: 0 = energy, 1 = species (Jacobi), 2 = pressure
// (multigrid when enabled, Jacobi otherwise).
int cg_solve64(ds_grid* g, int sys, double sc, double* x, hipStream_t s, int* iters, double* res, double tol) {
  int st;
  g->f32_sys = -1;
  Lev<double> L = g->L0;
  L.sc = sc;
  L.qc = g->qc;
  L.diag = g->diag;
  pressure_type(g, sys, L);
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
    CgVecs<double> V{x, g->r, g->pd, g->p_alt, g->q, H ? nullptr : g->zj};
    if (sys != 2 && g->tune.neumann) V.r_alt = g->r_alt;
    double* const p_odd = V.p_alt;   // direction of odd iterations (for the deferred x update)
    double* const p_even = V.p;
    double* z = nullptr;
    cg_start(L, H, V, &z, ss, g->partials, g->counters + CT_SOLVE0, s);
    bool first = true;
    const bool timed = g->timing && H;
    while (!g->h_status[sys].done) {
      const int it0 = g->h_status[sys].it;
      const int b = batch_size(batch_of(g, sys, x), first);
      const int m = timed ? std::min(b, (int)ds_grid::NEV) : b;
      for (int t = 0; t < m; ++t) {
        cg_iteration(L, H, V, &z, ss, g->partials, g->counters + CT_SOLVE0, first, s,
                     timed ? g->ev[2 * t] : nullptr, timed ? g->ev[2 * t + 1] : nullptr);
        first = false;
      }
      HIPCHK(g, hipGetLastError());
      if ((st = sync_status(g, sys, s)) != DS_OK) return st;
      if (timed) accumulate_timing(g, g->h_status[sys].it - it0,
                                   ((L.dfly ? 40.0 : 48.0) + (cg_defers_x(L) ? 16.0 : 0.0)) * (double)g->n);
    }
    const int it = g->h_status[sys].it;
    if (it > 0 && cg_defers_x(L)) launch_axpy_alpha(x, (it & 1) ? p_odd : p_even, ss, g->n, s);
  }
  const SolveStatus& h = g->h_status[sys];
  batch_of(g, sys, x) = std::max(2, std::min(256, h.it));
  *iters = h.it;
  *res = h.res;
  if (sys == 2) g->diag_out.refinements_p = 0;
  return h.done == 1 ? DS_OK : DS_ERR_NOT_CONVERGED;
}

// The FP64 form's multigrid pressure solve in flight on a set of pressure
// arrays (as Mg32Run for the precision form): cg64p_begin enqueues the start
// and the first batch of iterations without a host test (the CG and V-cycle
// kernels read the device status and return at once once it has converged),
// cg64p_end takes the host tests and applies the last deferred update.
struct Cg64Run {
  Lev<double> L;
  MgHier<double>* H = nullptr;
  CgVecs<double> V{};
  double* z = nullptr;
  SolveStatus* ss = nullptr;
  const PBufs* B = nullptr;
  double* x = nullptr;
  hipStream_t s = nullptr;
  bool first = true;
  double *p_odd = nullptr, *p_even = nullptr;   // directions of odd and even iterations
};

int cg64p_batch(ds_grid* g, Cg64Run& R) {
  const int m = batch_size(batch_of(g, 2, R.x), R.first);
  for (int t = 0; t < m; ++t) {
    cg_iteration(R.L, R.H, R.V, &R.z, R.ss, R.B->partials, R.B->counters + CT_SOLVE0, R.first, R.s, nullptr,
                 nullptr);
    R.first = false;
  }
  HIPCHK(g, hipGetLastError());
  return DS_OK;
}

int cg64p_begin(ds_grid* g, const PBufs& B, double sc, double* x, hipStream_t s, double tol, Cg64Run& R) {
  int st;
  Lev<double> L = g->L0;
  L.sc = sc;
  L.qc = B.qc;
  L.diag = B.diag;
  pressure_type(g, 2, L);
  MgHier<double>& H = g->H64;
  H.lev[0] = L;
  mg_setup_levels(H, g->dirmask, s);
  SolveStatus* ss = g->status + 2;
  if ((st = init_status(g, 2, tol, g->prm.maxit, s)) != DS_OK) return st;
  launch_resid64(L, B.b, x, B.r, ss, B.partials, B.counters + CT_SOLVE0, true, s);
  launch_zero_if_flagged(x, g->n, ss, s);
  HIPCHK(g, hipGetLastError());
  g->h_status[2].done = 0;
  R.L = L;
  R.H = &H;
  R.V = CgVecs<double>{x, B.r, B.pd, B.p_alt, B.q, nullptr};
  R.z = nullptr;
  R.ss = ss;
  R.B = &B;
  R.x = x;
  R.s = s;
  R.first = true;
  R.p_odd = R.V.p_alt;
  R.p_even = R.V.p;
  cg_start(L, &H, R.V, &R.z, ss, B.partials, B.counters + CT_SOLVE0, s);
  return cg64p_batch(g, R);
}

int cg64p_end(ds_grid* g, Cg64Run& R, int* iters, double* res) {
  int st;
  if ((st = sync_status(g, 2, R.s)) != DS_OK) return st;
  while (!g->h_status[2].done) {
    if ((st = cg64p_batch(g, R)) != DS_OK) return st;
    if ((st = sync_status(g, 2, R.s)) != DS_OK) return st;
  }
  const int it = g->h_status[2].it;
  if (it > 0 && cg_defers_x(R.L)) launch_axpy_alpha(R.x, (it & 1) ? R.p_odd : R.p_even, R.ss, g->n, R.s);
  HIPCHK(g, hipGetLastError());
  const SolveStatus& h = g->h_status[2];
  batch_of(g, 2, R.x) = std::max(2, std::min(256, h.it));
  *iters = h.it;
  *res = h.res;
  g->diag_out.refinements_p = 0;
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
  pressure_type(g, sys, L);
  Lev<float> F;
  lev_dims(F, L.nx, L.ny, L.nz, sc);
  F.qc = g->qc32;
  F.diag = g->diag32;
  const bool mg = sys == 2 && g->prm.pressure_precond == 1;
  if (!take_f32(g, sys)) {
    launch_to_float(g->qc, g->qc32, g->n, s);
    if (mg) launch_mg_diag(F, g->dirmask, g->diag32, s);   // the formula the V-cycle forms on the fly
    else launch_to_float(g->diag, g->diag32, g->n, s);
  }
  MgHier<float>* H = nullptr;
  if (mg) {
    H = &g->H32;
    H->lev[0] = F;
    mg_setup_levels(*H, g->dirmask, s);
  }
  SolveStatus* so = g->status + sys;
  SolveStatus* si = g->status + 3;
  const int max_rounds = 12;
  if ((st = init_status(g, sys, tol, g->prm.maxit, s)) != DS_OK) return st;
  launch_resid64(L, g->b, x, g->r, so, g->partials, g->counters + CT_SOLVE0, true, s);
  launch_zero_if_flagged(x, g->n, so, s, g->r);   // r too: a round may start without a host test
  HIPCHK(g, hipGetLastError());
  // Energy and species on vectorised levels (one host test per round, below):
  // no host test of the start either; the first round's inner tolerance is
  // formed on the device from the start's residual.  A start that already
  // meets the tolerance then takes one round that only lowers the residual.
  const bool one_test = g->tune.round_test && sys != 2 && !H && cg_defers_x(F);
  if (one_test) g->h_status[sys].done = 0;
  else if ((st = sync_status(g, sys, s)) != DS_OK) return st;
  int total = 0, rounds = 0, inner_fail = 0;
  while (!g->h_status[sys].done && rounds < max_rounds && !inner_fail) {
    // Ask the FP32 solve for the reduction still needed (with a margin), but
    // not below what FP32 arithmetic reliably attains.
    const double floor = H || sys == 2 ? g->tune.inner_min : g->tune.inner_min_jac;
    if (one_test && rounds == 0) {
      launch_init_inner_status(si, so, 0.5 * tol, floor, 0.5, g->prm.maxit, s);
    } else {
      const double need = 0.5 * tol / std::max(g->h_status[sys].res, 1e-300);
      const double inner_tol = std::min(0.5, std::max(floor, need));
      if ((st = init_status(g, 3, inner_tol, g->prm.maxit, s)) != DS_OK) return st;
    }
    g->h_status[3].it = 0;
    g->h_status[3].done = 0;
    CgVecs<float> V{g->e32, g->r32, g->p32, g->p32alt, g->q32, H ? nullptr : g->zj32};
    if (sys != 2 && g->tune.neumann) V.r_alt = g->r32alt;
    float* const p_odd = V.p_alt;   // direction of odd iterations (for the deferred x update)
    float* const p_even = V.p;
    float* z = nullptr;
    // Jacobi rounds on vectorised levels: conversion, z = r/diag and both
    // dot products in one pass (the Neumann-polynomial z then in a marching
    // pass of its own); otherwise the conversion, then cg_start
    if (!H && V.r_alt && launch_inner_init_jac<float>(F, g->r, g->r32, g->e32, nullptr, si, g->partials,
                                                      g->counters + CT_SOLVE1, s)) {
      launch_neumann_start<float>(F, V.r, V.zj, si, g->partials, g->counters + CT_SOLVE0 + 2, s);
    } else if (H || !launch_inner_init_jac<float>(F, g->r, g->r32, g->e32, g->zj32, si, g->partials,
                                                 g->counters + CT_SOLVE1, s)) {
      launch_inner_init<float>(F, g->r, g->r32, g->e32, si, g->partials, g->counters + CT_SOLVE1, s);
      cg_start(F, H, V, &z, si, g->partials, g->counters + CT_SOLVE0, s);
    }
    bool first = true;
    const bool timed = g->timing && H;
    int& expect = g->batch_round[sys][std::min(rounds, 2)];
    // Energy and species (diagonally dominant, a few inner iterations per
    // round) on vectorised levels: the round's inner iterations
    // are enqueued without a host test (the expected count plus one; each
    // returns at once after convergence), the correction takes the last
    // deferred direction by the device's iteration count, and the round's one
    // host test reads the inner and outer statuses together.  A round whose
    // inner solve stopped short only reduces the residual less: the next
    // round goes on from there.
    if (one_test) {
      const int m = batch_size(expect + 1, true);
      for (int t = 0; t < m; ++t) {
        cg_iteration(F, H, V, &z, si, g->partials, g->counters + CT_SOLVE0, first, s);
        first = false;
      }
      launch_add_correction_by_parity(F, x, g->e32, p_even, p_odd, si, s);
      launch_resid64(L, g->b, x, g->r, so, g->partials, g->counters + CT_SOLVE0, false, s);
      HIPCHK(g, hipGetLastError());
      if ((st = sync_status2(g, 3, sys, s)) != DS_OK) return st;
      const SolveStatus& hs = g->h_status[3];
      total += hs.it;
      expect = hs.done ? std::max(2, std::min(256, hs.it)) : std::min(256, 2 * hs.it);
      inner_fail = hs.done == 2;
      ++rounds;
      continue;
    }
    do {
      const int it0 = g->h_status[3].it;
      // one iteration of margin for the Jacobi-type systems: an iteration
      // that finds the solve converged costs two launches that return at once,
      // well under one more host convergence test
      const int b = batch_size(H ? expect : expect + 1, first);
      const int m = timed ? std::min(b, (int)ds_grid::NEV) : b;
      for (int t = 0; t < m; ++t) {
        cg_iteration(F, H, V, &z, si, g->partials, g->counters + CT_SOLVE0, first, s,
                     timed ? g->ev[2 * t] : nullptr, timed ? g->ev[2 * t + 1] : nullptr);
        first = false;
      }
      HIPCHK(g, hipGetLastError());
      if ((st = sync_status(g, 3, s)) != DS_OK) return st;
      if (timed) accumulate_timing(g, g->h_status[3].it - it0, 24.0 * (double)g->n);
    } while (!g->h_status[3].done);
    // x += e, with the inner solve's last deferred e += alpha p folded in
    const int it = g->h_status[3].it;
    const float* p_last = (it > 0 && cg_defers_x(F)) ? ((it & 1) ? p_odd : p_even) : nullptr;
    total += g->h_status[3].it;
    expect = std::max(2, std::min(256, g->h_status[3].it));
    inner_fail = g->h_status[3].done == 2;
    launch_add_correction<float>(F, x, g->e32, s, p_last, si);
    launch_resid64(L, g->b, x, g->r, so, g->partials, g->counters + CT_SOLVE0, false, s);
    HIPCHK(g, hipGetLastError());
    if ((st = sync_status(g, sys, s)) != DS_OK) return st;
    ++rounds;
  }
  batch_of(g, sys, x) = std::max(2, std::min(256, total / std::max(1, rounds)));
  *iters = total;
  *res = g->h_status[sys].res;
  if (sys == 2) g->diag_out.refinements_p = rounds;
  else if (sys == 0) g->diag_out.rounds_T = rounds;
  else g->diag_out.rounds_omega = rounds;
  return g->h_status[sys].done == 1 ? DS_OK : DS_ERR_NOT_CONVERGED;
}

// The graph of two FP32-multigrid CG iterations for the current buffers and
// scale, captured on first use (null: capture failed; the caller then runs
// the iterations one by one and graphs are switched off for the handle).
hipGraphExec_t mg32_graph(ds_grid* g, const PBufs& B, const Lev<double>& L, MgHier<float>& H, const CgVecsMg32& V,
                          float* z, SolveStatus* st, double sc) {
  for (auto& e : g->graphs)
    if (e.ex && e.x == V.x && e.p == V.p && e.z == z && e.sc == sc) return e.ex;
  if (!g->cap_stream && hipStreamCreateWithFlags(&g->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    (void)hipGetLastError();
    g->cap_stream = nullptr;
    g->tune.graphs = 0;
    return nullptr;
  }
  hipGraphExec_t ex = capture_mg32_pair(L, H, V, B.r32, z, st, B.partials, B.counters + CT_SOLVE0, g->cap_stream);
  if (!ex) {
    g->tune.graphs = 0;
    return nullptr;
  }
  auto& e = g->graphs[g->graph_next];
  g->graph_next = (g->graph_next + 1) % ds_grid::NGRAPH;
  if (e.ex) (void)hipGraphExecDestroy(e.ex);
  e.ex = ex;
  e.x = V.x;
  e.p = V.p;
  e.z = z;
  e.sc = sc;
  return ex;
}

// One FP32-multigrid CG solve in flight: mg32_begin enqueues its start and
// its first batch of iterations without a host test (every kernel reads the
// device status and returns at once once the solve has converged); mg32_end
// takes the host tests, enqueues further batches until converged and applies
// the last deferred update.
struct Mg32Run {
  Lev<double> L;
  MgHier<float>* H = nullptr;
  CgVecsMg32 V{};
  float* z = nullptr;
  SolveStatus* ss = nullptr;
  const PBufs* B = nullptr;
  double sc = 0.0;
  double* x = nullptr;
  hipStream_t s = nullptr;
  bool first = true;
};

int mg32_batch(ds_grid* g, Mg32Run& R) {
  const PBufs& B = *R.B;
  const int m = batch_size(batch_of(g, 2, R.x), R.first);
  int t = 0;
  if (R.first) {
    cg_iteration_mg32(R.L, *R.H, R.V, B.r32, &R.z, R.ss, B.partials, B.counters + CT_SOLVE0, true, R.s);
    R.first = false;
    ++t;
  }
  hipGraphExec_t ex = nullptr;
  for (; g->tune.graphs && t + 2 <= m; t += 2) {
    if (!ex && !(ex = mg32_graph(g, B, R.L, *R.H, R.V, R.z, R.ss, R.sc))) break;
    HIPCHK(g, hipGraphLaunch(ex, R.s));
  }
  for (; t < m; ++t) cg_iteration_mg32(R.L, *R.H, R.V, B.r32, &R.z, R.ss, B.partials, B.counters + CT_SOLVE0, false, R.s);
  HIPCHK(g, hipGetLastError());
  return DS_OK;
}

// f32_ready: the setup wrote B's FP32 copies of the operator.
int mg32_begin(ds_grid* g, const PBufs& B, bool f32_ready, double sc, double* x, hipStream_t s, double tol,
               Mg32Run& R) {
  int st;
  const int sys = 2;
  Lev<double> L = g->L0;
  L.sc = sc;
  L.qc = B.qc;
  L.diag = B.diag;
  pressure_type(g, sys, L);
  const bool phi = g->phi_op;   // the potential, on its own operator arrays
  if (phi) L.qc = g->phi_qc;
  Lev<float> F;
  lev_dims(F, L.nx, L.ny, L.nz, sc);
  F.qc = phi ? g->phi_q[0] : B.qc32;
  F.diag = phi ? g->phi_d[0] : B.diag32;
  // the value phi_q[0] holds in every cell: 1/dt rounded to FP32, as the setup's q converted
  if (phi && g->tune.const_q) F.qk = (float)(1.0 / g->dp.dt);
  if (phi && g->tune.const_q) L.qk = 1.0 / g->dp.dt;   // and in FP64, the value phi_qc holds
  if (phi) {
    if (!g->phi_ready) {
      launch_to_float(g->phi_qc, g->phi_q[0], g->n, s);
      launch_mg_diag(F, g->dirmask, g->phi_d[0], s);
      g->H32phi = g->H32;
      for (int l = 1; l < g->H32phi.nlev; ++l) {
        g->H32phi.lev[l].qc = g->phi_q[l];
        g->H32phi.lev[l].diag = g->phi_d[l];
      }
    }
  } else if (!f32_ready) {
    launch_to_float(B.qc, B.qc32, g->n, s);
    launch_mg_diag(F, g->dirmask, B.diag32, s);   // the formula the V-cycle forms on the fly
  }
  MgHier<float>& H = phi ? g->H32phi : g->H32;
  H.lev[0] = F;
  if (phi && g->phi_ready) {
    for (int l = 0; l < H.nlev; ++l) {   // the coarse levels are built already
      H.lev[l].dfly = 1;
      H.lev[l].dmask = g->dirmask;
    }
  } else {
    mg_setup_levels(H, g->dirmask, s);
  }
  if (phi) g->phi_ready = true;
  SolveStatus* ss = g->status + sys;
  if ((st = init_status(g, sys, tol, g->prm.maxit, s)) != DS_OK) return st;
  launch_resid64(L, B.b, x, B.r, ss, B.partials, B.counters + CT_SOLVE0, true, s, B.r32);
  launch_zero_if_flagged(x, g->n, ss, s);
  HIPCHK(g, hipGetLastError());
  g->h_status[sys].done = 0;
  R.L = L;
  R.H = &H;
  R.V = CgVecsMg32{x, B.r, B.p32, B.p32alt, B.q};   // iteration t writes its direction into p_alt (t odd) or p
  R.z = nullptr;
  R.ss = ss;
  R.B = &B;
  R.sc = sc;
  R.x = x;
  R.s = s;
  R.first = true;
  cg_start_mg32(L, H, B.r, B.r32, &R.z, ss, B.partials, B.counters + CT_SOLVE0, s, true);
  return mg32_batch(g, R);
}

int mg32_end(ds_grid* g, Mg32Run& R, int* iters, double* res) {
  int st;
  const int sys = 2;
  if ((st = sync_status(g, sys, R.s)) != DS_OK) return st;
  while (!g->h_status[sys].done) {
    if ((st = mg32_batch(g, R)) != DS_OK) return st;
    if ((st = sync_status(g, sys, R.s)) != DS_OK) return st;
  }
  const int it = g->h_status[sys].it;
  if (it > 0) launch_axpy_alpha(R.x, (it & 1) ? R.V.p_alt : R.V.p, R.ss, g->n, R.s);
  HIPCHK(g, hipGetLastError());
  const SolveStatus& h = g->h_status[sys];
  batch_of(g, sys, R.x) = std::max(2, std::min(256, h.it));
  *iters = h.it;
  *res = h.res;
  g->diag_out.refinements_p = 0;
  return h.done == 1 ? DS_OK : DS_ERR_NOT_CONVERGED;
}

// Precision form of a multigrid-preconditioned solve: FP64 conjugate
// gradients (operator, vectors, dot products) with the V-cycle -- the bulk of
// each iteration's memory traffic -- in FP32 on FP32 copies of the operator.
// No restarts: the FP64 recurrence converges to tol like cg_solve64.  On the
// shared arrays (pb[0]).
int cg_solve64_mg32(ds_grid* g, double sc, double* x, hipStream_t s, int* iters, double* res, double tol) {
  const bool f32_ready = !g->phi_op && take_f32(g, 2);
  if (g->phi_op) g->f32_sys = -1;
  Mg32Run R;
  int st = mg32_begin(g, g->pb[0], f32_ready, sc, x, s, tol, R);
  if (st != DS_OK) return st;
  return mg32_end(g, R, iters, res);
}

int solve(ds_grid* g, int sys, double sc, double* x, hipStream_t s, int* iters, double* res, double tol) {
  if (g->prm.precision == DS_PREC_MIXED) {
    if (sys == 2 && g->prm.pressure_precond == 1 && g->tune.mg32 && mg32_supported(g->L0))
      return cg_solve64_mg32(g, sc, x, s, iters, res, tol);
    return cg_solve_mixed(g, sys, sc, x, s, iters, res, tol);
  }
  return cg_solve64(g, sys, sc, x, s, iters, res, tol);
}
int solve(ds_grid* g, int sys, double sc, double* x, hipStream_t s, int* iters, double* res) {
  return solve(g, sys, sc, x, s, iters, res, g->prm.tol);
}

// The liquid-transport potential: x = A^-1 b with b in g->b.  By the direct
// solve where the grid allows it (then its operator arrays come from the
// setup's qc and diag, and the true FP64 residual is checked: iterations 0);
// otherwise, or should that residual miss tol, the multigrid CG from there.
// own: the setup wrote the precision form's own operator arrays of the
// potential instead of qc and diag (the CG path only).
int solve_potential(ds_grid* g, double* x, hipStream_t s, int* iters, double* res, double tol, bool own) {
  const DevParams& P = g->dp;
  const double sc = P.dt / (P.h * P.h);
  if (g->tune.phi_direct && g->fdm_ok && !own) {
    if (launch_fdm_solve(P, sc * (1.0 / P.dt), g->b, x, g->pd, s) == 0) {
      Lev<double> L = g->L0;
      L.sc = sc;
      L.qc = g->qc;
      L.diag = g->diag;
      L.qk = 1.0 / P.dt;   // the value qc holds in every cell
      pressure_type(g, 2, L);
      int st;
      if ((st = init_status(g, 2, tol, g->prm.maxit, s)) != DS_OK) return st;
      launch_resid64(L, g->b, x, g->r, g->status + 2, g->partials, g->counters + CT_SOLVE0, true, s, nullptr, true);
      HIPCHK(g, hipGetLastError());
      if ((st = sync_status(g, 2, s)) != DS_OK) return st;
      if (g->h_status[2].done == 1) {
        *iters = 0;
        *res = g->h_status[2].res;
        return DS_OK;
      }
    }
  }
  g->phi_op = own;
  const int st = solve(g, 2, sc, x, s, iters, res, tol);
  g->phi_op = false;
  return st;
}
// Does the potential take the direct solve (its setup then writes qc and diag)?
bool potential_direct(const ds_grid* g) { return g->tune.phi_direct && g->fdm_ok; }

int solve_pressure_system(ds_grid* g, hipStream_t s, int* iters, double* res) {
  const DevParams& P = g->dp;
  return solve(g, 2, P.dt / (P.h * P.h), g->p, s, iters, res);
}

int evaporation_source(ds_grid* g, hipStream_t s) {
  const DevParams& P = g->dp;
  if (P.evaporation) {
    // literal species form: the liquid holds omega_sat(T) before the flux reads omega
    if (P.species_form == DS_SPECIES_LITERAL) launch_liquid_saturation(P, g->alpha, g->T, g->omega, g->c, g->band, g->band_count, s);
    launch_interface(P, g->alpha, g->T, g->omega, g->u, g->v, g->w, g->mraw, g->adj, g->band, g->band_count, g->partials,
                     g->counters + CT_IFACE, g->scal, s);
  } else {
    launch_fill(g->mraw, 0.0, g->n, s);
    launch_fill(g->scal + SC_K, 0.0, 4, s);
  }
  launch_source(P, g->alpha, g->mraw, g->scal, g->mdot, g->a1, s);
  HIPCHK(g, hipGetLastError());
  return DS_OK;
}

// Implicit viscous momentum on (us, vs, ws) in place (eqs. 5 and 30), with
// alpha' in a_new: Jacobi-PCG over the concatenated faces, batches of
// iterations between host convergence tests (the status slot of the energy
// solve, which is done by then).  P: the stage's parameters (its gas density).
int viscous_solve(ds_grid* g, const double* a_new, hipStream_t s, int* iters, double* res, const DevParams& P) {
  SolveStatus* ss = g->status + 0;
  int st;
  if ((st = init_status(g, 0, g->prm.tol, g->prm.maxit, s)) != DS_OK) return st;
  launch_visc_start(P, a_new, g->us, g->vs, g->ws, g->u, g->v, g->w, g->visc, ss, g->partials,
                    g->counters + CT_SOLVE1, s);
  HIPCHK(g, hipGetLastError());
  g->h_status[0].done = 0;
  bool first = true;
  while (!g->h_status[0].done) {
    const int m = batch_size(g->batch_visc, first);
    first = false;
    for (int t = 0; t < m; ++t) launch_visc_iteration(P, a_new, g->visc, ss, g->partials, g->counters + CT_SOLVE1, s);
    HIPCHK(g, hipGetLastError());
    if ((st = sync_status(g, 0, s)) != DS_OK) return st;
  }
  launch_visc_store(P, g->visc, g->us, g->vs, g->ws, s);
  HIPCHK(g, hipGetLastError());
  const SolveStatus& h = g->h_status[0];
  g->batch_visc = std::max(2, std::min(256, h.it));
  *iters = h.it;
  *res = h.res;
  return h.done == 1 ? DS_OK : DS_ERR_NOT_CONVERGED;
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
  // The second stream (where the pressure has arrays of its own): forked from s with an event and joined back
  // into s with another, on every return path too.
  if (g->pb_own && !g->s2 && !g->s2_failed) {
    if (hipStreamCreateWithFlags(&g->s2, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      g->s2_failed = true;
    }
  }
  const bool overlap = g->pb_own && !g->timing && !g->s2_failed;
  struct Join {
    ds_grid* g;
    hipStream_t s;
    bool on = false;
    ~Join() {
      if (on) {
        (void)hipEventRecord(g->ev_join, g->s2);
        (void)hipStreamWaitEvent(s, g->ev_join, 0);
      }
    }
  } join{g, s};
  auto fork = [&]() -> int {
    HIPCHK(g, hipEventRecord(g->ev_fork, s));
    HIPCHK(g, hipStreamWaitEvent(g->s2, g->ev_fork, 0));
    join.on = true;
    return DS_OK;
  };
  auto join_now = [&]() -> int {
    HIPCHK(g, hipEventRecord(g->ev_join, g->s2));
    HIPCHK(g, hipStreamWaitEvent(s, g->ev_join, 0));
    join.on = false;
    return DS_OK;
  };
  // 3 (first part).  The liquid-transport potential reads only u^n: by the direct solve it runs on the second
  // stream (on the pressure's own arrays, their A p array as the transforms' scratch) while the evaporation and
  // liquid sources run on s.  Its residual check takes the constant coefficient 1/dt from its value (no
  // operator arrays written or read) and keeps only the status (no residual array) where the marching
  // residual kernel runs; the multigrid CG that would take over on s sets up its own.
  const bool phi_fork = overlap && g->prm.liquid_transport && potential_direct(g);
  if (phi_fork) {
    const PBufs& B = g->pb[1];
    const double sc = P.dt / (P.h * P.h);
    Lev<double> L = g->L0;
    L.sc = sc;
    L.qc = B.qc;
    L.diag = B.diag;
    L.qk = 1.0 / P.dt;
    pressure_type(g, 2, L);
    const bool cq = resid64_cq_ok(L);
    if ((st = fork()) != DS_OK) return st;
    launch_div_setup(P, g->u, g->v, g->w, cq ? nullptr : B.qc, cq ? nullptr : B.diag, B.b, g->s2);
    if (launch_fdm_solve(P, sc * (1.0 / P.dt), B.b, g->phi, B.q, g->s2) != 0)
      return fail(g, DS_ERR_STATE, "internal: the direct potential solve refused the grid");
    if ((st = init_status(g, 2, g->prm.tol_phi, g->prm.maxit, g->s2)) != DS_OK) return st;
    launch_resid64(L, B.b, g->phi, cq ? nullptr : B.r, g->status + 2, B.partials, B.counters + CT_SOLVE0, true,
                   g->s2, nullptr, cq);
    HIPCHK(g, hipGetLastError());
  }
  // 1-2. evaporation source and liquid source
  if ((st = evaporation_source(g, s)) != DS_OK) return st;
  bool phi_done = false;
  if (phi_fork) {
    if ((st = sync_status(g, 2, g->s2)) != DS_OK) return st;
    if ((st = join_now()) != DS_OK) return st;
    if (g->h_status[2].done == 1) {
      D.iters_phi = 0;
      D.res_phi = g->h_status[2].res;
      phi_done = true;
    }
    // otherwise the path below solves again on s (the multigrid CG from the direct solve's result)
  }
  // 3. advection of alpha1 with the divergence-free part of u^n, c and T with u^n
  if (g->prm.liquid_transport && !phi_done) {
    // precision form, multigrid: the potential's own operator arrays, written by its first setup only
    const bool own = !potential_direct(g) && g->prm.precision == DS_PREC_MIXED && g->prm.pressure_precond == 1 &&
                     g->tune.mg32 && mg32_supported(g->L0);
    if (own) launch_div_setup(P, g->u, g->v, g->w, g->phi_ready ? nullptr : g->phi_qc, g->diag, g->b, s);
    else if (potential_direct(g)) launch_div_setup(P, g->u, g->v, g->w, g->qc, g->diag, g->b, s);
    else launch_div_setup(P, g->u, g->v, g->w, g->qc, g->diag, g->b, s, f32_out(g, 2));
    st = solve_potential(g, g->phi, s, &D.iters_phi, &D.res_phi, g->prm.tol_phi, own);
    if (st == DS_ERR_NOT_CONVERGED) rc = st;
    else if (st != DS_OK) return st;
  } else if (!g->prm.liquid_transport) {
    D.iters_phi = 0;
    D.res_phi = 0.0;
  }
  const bool var = g->prm.gas_density == DS_GAS_VARIABLE;
  // geometric advection: the liquid fluxes of every face from the planes of the surface cells
  const bool geo = g->prm.advection == DS_ADV_GEOMETRIC;
  if (geo) {
    double* const pl[4] = {g->geo_pl[0], g->geo_pl[1], g->geo_pl[2], g->geo_pl[3]};
    launch_geo_fluxes(P, g->a1, g->u, g->v, g->w, g->prm.liquid_transport ? g->phi : nullptr, pl, g->geo_F[0],
                      g->geo_F[1], g->geo_F[2], s);
  }
  const double* Fx = geo ? g->geo_F[0] : nullptr;
  const double* Fy = geo ? g->geo_F[1] : nullptr;
  const double* Fz = geo ? g->geo_F[2] : nullptr;
  if (var) {
    // the vapour flux carries the face value of rho_G omega (start-of-step rho_G)
    launch_gas_partial(P, g->omega, g->rg, g->qv, s);
    DevParams Pa = P;
    Pa.rho_G = 1.0;
    Pa.rg = nullptr;
    launch_advect(Pa, g->a1, g->qv, g->T, g->c, g->u, g->v, g->w, g->prm.liquid_transport ? g->phi : nullptr,
                  g->a_new, g->c_new, g->T_new, g->partials, g->counters + CT_ADV, g->scal, s, Fx, Fy, Fz);
    // rho_G' of the advected state (T', c', alpha')
    launch_gas_invert(P, P.solve_energy ? g->T_new : g->T, g->c_new, g->a_new, g->rg_p, s);
  } else {
    launch_advect(P, g->a1, g->omega, g->T, g->c, g->u, g->v, g->w, g->prm.liquid_transport ? g->phi : nullptr,
                  g->a_new, g->c_new, g->T_new, g->partials, g->counters + CT_ADV, g->scal, s, Fx, Fy, Fz);
  }
  // stages after the advection read rho_G' (a variable gas)
  DevParams Pp = P;
  if (var) Pp.rg = g->rg_p;
  // The predictor and the pressure (5c, 6) read none of what the energy and species stages write, nor write
  // what they read: with the pressure's own arrays they run on the second stream, forked here and joined
  // before the projection (on every return path).
  const bool mixed = g->prm.precision == DS_PREC_MIXED;
  Mg32Run PR;
  Cg64Run PR64;
  if (overlap) {
    if ((st = fork()) != DS_OK) return st;
    const PBufs& B = g->pb[1];
    launch_predictor(Pp, g->a_new, g->xi, g->u, g->v, g->w, g->us, g->vs, g->ws, g->s2);
    launch_pressure_setup(Pp, g->a_new, g->mdot, g->us, g->vs, g->ws, B.qc, B.diag, B.b, g->s2,
                          mixed ? f32_out_own(g) : F32Out{}, nullptr);
    const double sc = P.dt / (P.h * P.h);
    st = mixed ? mg32_begin(g, B, true, sc, g->p, g->s2, g->prm.tol, PR)
               : cg64p_begin(g, B, sc, g->p, g->s2, g->prm.tol, PR64);
    if (st != DS_OK) return st;
  }
  // 5a. energy (warm start T')
  if (P.solve_energy) {
    launch_energy_setup(Pp, g->a_new, g->T_new, g->mdot, g->u, g->v, g->w, g->qc, g->diag, g->b, s,
                        f32_out(g, 0));
    st = solve(g, 0, 1.0 / (P.h * P.h), g->T_new, s, &D.iters_T, &D.res_T);
    if (st == DS_ERR_NOT_CONVERGED) rc = st;
    else if (st != DS_OK) return st;
    std::swap(g->T, g->T_new);
  } else {
    D.iters_T = 0;
    D.res_T = 0.0;
    D.rounds_T = 0;
  }
  // 5b. species (warm start omega' = c'/(rho_G theta))
  const bool extrap = g->tune.extrap && !g->recording;
  launch_species_setup(Pp, g->a_new, g->c_new, g->mdot, g->u, g->v, g->w, g->qc, g->diag, g->b, g->om_new, s,
                       f32_out(g, 1), extrap && g->corr_ok ? g->om_corr : nullptr);
  st = solve(g, 1, (var ? 1.0 : P.rho_G) * P.D / (P.h * P.h), g->om_new, s, &D.iters_omega, &D.res_omega);
  if (st == DS_ERR_NOT_CONVERGED) rc = st;
  else if (st != DS_OK) return st;
  launch_species_update(Pp, g->a_new, g->c_new, g->mdot, g->om_new, g->u, g->v, g->w, g->c, g->omega,
                        g->partials, g->counters + CT_SPEC, g->scal, s, extrap ? g->om_corr : nullptr);
  g->corr_ok = extrap;
  // a variable gas: (omega, rho_G) of the new state from (T, c), and eq. 7's compressibility term
  if (var) launch_gas_end(P, g->T, g->c, g->a_new, g->rg_p, g->omega, g->rg, g->scomp, s);
  if (overlap) {
    D.iters_visc = 0;
    D.res_visc = 0.0;
    st = mixed ? mg32_end(g, PR, &D.iters_p, &D.res_p) : cg64p_end(g, PR64, &D.iters_p, &D.res_p);
    if (st == DS_ERR_NOT_CONVERGED) rc = st;
    else if (st != DS_OK) return st;
  } else {
    // 5c. momentum predictor with alpha' (and its implicit viscous part)
    launch_predictor(Pp, g->a_new, g->xi, g->u, g->v, g->w, g->us, g->vs, g->ws, s);
    if (P.viscous) {
      st = viscous_solve(g, g->a_new, s, &D.iters_visc, &D.res_visc, Pp);
      if (st == DS_ERR_NOT_CONVERGED) rc = st;
      else if (st != DS_OK) return st;
    } else {
      D.iters_visc = 0;
      D.res_visc = 0.0;
    }
    // 6. pressure (warm start p^n) and correction
    launch_pressure_setup(Pp, g->a_new, g->mdot, g->us, g->vs, g->ws, g->qc, g->diag, g->b, s, f32_out(g, 2),
                          var ? g->scomp : nullptr);
    st = solve_pressure_system(g, s, &D.iters_p, &D.res_p);
    if (st == DS_ERR_NOT_CONVERGED) rc = st;
    else if (st != DS_OK) return st;
  }
  if (join.on && (st = join_now()) != DS_OK) return st;   // the projection reads p and u* from the second stream
  // 7. projection, and the diagnostics of the new state (alpha = alpha') in the same pass
  launch_project_diagnostics(Pp, g->a_new, g->p, g->us, g->vs, g->ws, g->u, g->v, g->w, g->c, g->T, g->mdot,
                             g->partials, g->counters + CT_DIAG, g->scal, s);
  std::swap(g->alpha, g->a_new);
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

// ---------------------------------------------------------------- differentiation form
int save_slot(ds_grid* g, const Slot& sl, hipStream_t s) {
  const size_t nb = g->n * sizeof(double);
  const std::pair<double*, const double*> cp[7] = {{sl.alpha, g->alpha}, {sl.c, g->c},   {sl.omega, g->omega},
                                                   {sl.T, g->T},         {sl.p, g->p},   {sl.phi, g->phi},
                                                   {sl.omt, g->om_new}};
  for (const auto& q : cp) HIPCHK(g, hipMemcpyAsync(q.first, q.second, nb, hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(sl.u, g->u, g->nu * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(sl.v, g->v, g->nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(sl.w, g->w, g->nw * sizeof(double), hipMemcpyDeviceToDevice, s));
  return DS_OK;
}

int load_slot(ds_grid* g, const Slot& sl, hipStream_t s) {
  const size_t nb = g->n * sizeof(double);
  const std::pair<double*, const double*> cp[7] = {{g->alpha, sl.alpha}, {g->c, sl.c},     {g->omega, sl.omega},
                                                   {g->T, sl.T},         {g->p, sl.p},     {g->phi, sl.phi},
                                                   {g->om_new, sl.omt}};
  for (const auto& q : cp) HIPCHK(g, hipMemcpyAsync(q.first, q.second, nb, hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(g->u, sl.u, g->nu * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(g->v, sl.v, g->nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipMemcpyAsync(g->w, sl.w, g->nw * sizeof(double), hipMemcpyDeviceToDevice, s));
  return DS_OK;
}

// d rho_G / d T_amb of eq. 24 (ideal gas, or the Peng-Robinson Z of the
// ambient gas by the implicit-function rule on its cubic).
double host_drhoG_dT(const ds_params& q, double rho_G) {
  const double T = q.T_amb;
  if (q.eq_model != DS_EQ_PENG_ROBINSON) return -rho_G / T;
  const double Z = host_pr_Z(T, q.p, q.Tc_G, q.Pc_G, q.acentric_G);
  const double kap = 0.37464 + 1.54226 * q.acentric_G - 0.26992 * q.acentric_G * q.acentric_G;
  const double K0 = 0.45724 * R_GAS * R_GAS * q.Tc_G * q.Tc_G / q.Pc_G;
  const double sq = 1.0 + kap * (1.0 - std::sqrt(T / q.Tc_G));
  const double a = K0 * sq * sq;
  const double da = 2.0 * K0 * sq * (-kap / (2.0 * std::sqrt(T * q.Tc_G)));
  const double b = 0.07780 * R_GAS * q.Tc_G / q.Pc_G;
  const double A = a * q.p / (R_GAS * T * R_GAS * T), B = b * q.p / (R_GAS * T);
  const double dA = q.p / (R_GAS * R_GAS) * (da / (T * T) - 2.0 * a / (T * T * T));
  const double dB = -B / T;
  const double c2 = -(1.0 - B), c1 = A - 3.0 * B * B - 2.0 * B;
  const double FZ = (3.0 * Z + 2.0 * c2) * Z + c1;
  const double FA = Z - B;
  const double FB = Z * Z + (-6.0 * B - 2.0) * Z + (-A + 2.0 * B + 3.0 * B * B);
  const double dZ = -(FA * dA + FB * dB) / FZ;
  return -rho_G * (1.0 / T + dZ / Z);
}

// Adjoint solve A lam = b (b in g->b).  Adjoint right-hand sides can be
// tiny (far-field tails of alpha reach the box faces at 1e-150 and below),
// where the squared norms of conjugate gradients underflow; b is therefore
// scaled by a power of two (exactly) to a maximum in [1/2, 1) and lam scaled back.
int adj_solve(ds_grid* g, int sys, double sc, double tol, int slot, hipStream_t s, int* rc, bool potential = false) {
  launch_absmax(g->b, g->n, g->partials, g->counters + CT_ADJ, g->scal + SC_ABSMAX, s);
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipMemcpyAsync(g->h_scal + SC_ABSMAX, g->scal + SC_ABSMAX, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(g, hipStreamSynchronize(s));
  const double bmax = g->h_scal[SC_ABSMAX];
  launch_fill(g->lam, 0.0, g->n, s);
  if (bmax == 0.0) return DS_OK;
  if (!std::isfinite(bmax)) return fail(g, DS_ERR_NONFINITE, "non-finite adjoint right-hand side");
  int ex = 0;
  std::frexp(bmax, &ex);
  launch_scale(g->b, std::ldexp(1.0, -ex), g->n, s);
  int it = 0;
  double res = 0.0;
  const int st = potential ? solve_potential(g, g->lam, s, &it, &res, tol, false) : solve(g, sys, sc, g->lam, s, &it, &res, tol);
  g->adj_iters[slot] += it;
  if (st == DS_ERR_NOT_CONVERGED) *rc = st;
  else if (st != DS_OK) return st;
  launch_scale(g->lam, std::ldexp(1.0, ex), g->n, s);
  HIPCHK(g, hipGetLastError());
  return DS_OK;
}

// Reverse of one step: replay the explicit stages of the step from `cur`
// (the solves' results come from `nxt`), then apply the transposed stages in
// reverse order to the adjoint state held in A_al, A_c, A_om, A_T, A_U.
int reverse_step(ds_grid* g, const Slot& cur, const Slot& nxt, hipStream_t s, int* rc) {
  const DevParams& P = g->dp;
  int st;
  unsigned* cadj = g->counters + CT_ADJ;
  // replay: interface source, liquid source, advection, predictor
  if (P.evaporation) {
    launch_interface(P, cur.alpha, cur.T, cur.omega, cur.u, cur.v, cur.w, g->mraw, g->adj, g->band, g->band_count, g->partials,
                     g->counters + CT_IFACE, g->scal, s);
  } else {
    launch_fill(g->mraw, 0.0, g->n, s);
    launch_fill(g->scal + SC_K, 0.0, 4, s);
  }
  launch_source(P, cur.alpha, g->mraw, g->scal, g->mdot, g->a1, s);
  const double* phi = g->prm.liquid_transport ? nxt.phi : nullptr;
  launch_advect(P, g->a1, cur.omega, cur.T, cur.c, cur.u, cur.v, cur.w, phi, g->a_new, g->c_new, g->T_new,
                g->partials, g->counters + CT_ADV, g->scal, s);
  launch_predictor(P, g->a_new, g->xi, cur.u, cur.v, cur.w, g->us, g->vs, g->ws, s);
  HIPCHK(g, hipGetLastError());
  // projection and pressure (S11, S10)
  launch_pressure_setup(P, g->a_new, g->mdot, g->us, g->vs, g->ws, g->qc, g->diag, g->b, s);
  launch_adj_project(P, g->a_new, nxt.p, g->A_U, g->b, g->A_ab, g->partials, cadj, g->grad, s);
  if ((st = adj_solve(g, 2, P.dt / (P.h * P.h), g->prm.tol, 0, s, rc)) != DS_OK) return st;
  launch_adj_pressure(P, g->a_new, nxt.p, g->lam, g->mdot, g->A_ab, g->A_md, g->partials, cadj, g->grad, s);
  // predictor (S9)
  launch_adj_predictor(P, g->a_new, g->xi, g->A_U, g->A_Us, g->Q, g->lam, cur.u, cur.v, cur.w, g->A_ab, g->partials,
                       cadj, g->grad, s);
  // species (S8)
  launch_species_setup(P, g->a_new, g->c_new, g->mdot, cur.u, cur.v, cur.w, g->qc, g->diag, g->b, nullptr, s);
  launch_adj_species_rhs(P, g->a_new, nxt.omt, g->A_om, g->A_c, g->b, g->A_ab, g->partials, cadj, g->grad, s);
  if ((st = adj_solve(g, 1, P.rho_G * P.D / (P.h * P.h), g->prm.tol, 1, s, rc)) != DS_OK) return st;
  launch_adj_species(P, g->a_new, nxt.omt, g->lam, cur.u, cur.v, cur.w, g->A_ab, g->A_cp, g->A_md, g->partials, cadj,
                     g->grad, s);
  // energy (S7)
  if (P.solve_energy) {
    launch_energy_setup(P, g->a_new, g->T_new, g->mdot, cur.u, cur.v, cur.w, g->qc, g->diag, g->b, s);
    HIPCHK(g, hipMemcpyAsync(g->b, g->A_T, g->n * sizeof(double), hipMemcpyDeviceToDevice, s));
    if ((st = adj_solve(g, 0, 1.0 / (P.h * P.h), g->prm.tol, 2, s, rc)) != DS_OK) return st;
    launch_adj_energy(P, g->a_new, g->T_new, nxt.T, g->lam, g->mdot, cur.u, cur.v, cur.w, g->A_ab, g->A_Tp, g->A_md,
                      g->partials, cadj, g->grad, s);
  }
  // advection (S5) and the liquid-transport potential
  launch_adj_advect(P, g->a1, cur.omega, cur.T, cur.u, cur.v, cur.w, phi, g->a_new, g->A_al, g->A_ab, g->A_cp,
                    g->A_Tp, g->A_U, g->A_Ul, g->A_a1, g->A_om, g->A_T, g->A_c, g->partials, cadj, g->grad, s);
  if (phi) {
    launch_div_setup(P, cur.u, cur.v, cur.w, g->qc, g->diag, g->b, s);
    launch_adj_phi_rhs(P, g->A_Ul, g->b, s);
    if ((st = adj_solve(g, 2, P.dt / (P.h * P.h), g->prm.tol_phi, 3, s, rc, true)) != DS_OK) return st;
    launch_adj_phi_faces(P, g->A_Ul, g->lam, g->A_U, s);
  }
  // liquid source, redistribution, interface flux (eq. 4, S4, S1-S3)
  launch_adj_source(P, cur.alpha, g->mraw, g->A_a1, g->A_md, g->A_al, g->scal, g->partials, cadj, g->grad, s);
  if (P.evaporation)
    launch_adj_interface(P, cur.alpha, cur.T, cur.omega, cur.u, cur.v, cur.w, g->mraw, g->adj, g->A_md, g->scal,
                         g->A_al, g->A_T, g->A_om, g->A_U, g->irec, g->partials, cadj, g->grad, s);
  HIPCHK(g, hipGetLastError());
  return DS_OK;
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
      prm->pressure_precond > 1 || prm->liquid_transport < 0 || prm->liquid_transport > 1 ||
      prm->species_form < 0 || prm->species_form > 1 || prm->viscous < 0 || prm->viscous > 1 ||
      prm->gas_density < 0 || prm->gas_density > 1 || prm->advection < 0 || prm->advection > 1 ||
      (prm->gas_density == DS_GAS_VARIABLE && prm->species_form == DS_SPECIES_LITERAL) ||
      (prm->viscous && (!(prm->mu_L >= 0.0) || !(prm->mu_G >= 0.0) || !std::isfinite(prm->mu_L) ||
                        !std::isfinite(prm->mu_G))))
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
  P.species_form = prm->species_form;
  P.viscous = prm->viscous;
  P.mu_L = prm->mu_L;
  P.mu_G = prm->mu_G;
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
  LaunchShape& sh = g->shape;
  if (const char* e = getenv("DSVOF_VEC_BLOCKS")) set_vec_max_blocks(sh, atoi(e));
  if (const char* e = getenv("DSVOF_VEC_YTILE")) sh.vec_ytile = atoi(e);
  if (const char* e = getenv("DSVOF_MARCH_THREADS")) set_march_threads(sh, atoi(e));
  if (const char* e = getenv("DSVOF_MARCH_MIN_PLANES")) set_march_min_planes(sh, atoi(e));
  for (int cls = 0; cls < 2; ++cls) {
    // DSVOF_MARCH_NT0 / DSVOF_MARCH_NT1: comma-separated block sizes, e.g. "512,256,384"
    const char* e = getenv(cls ? "DSVOF_MARCH_NT1" : "DSVOF_MARCH_NT0");
    if (!e) continue;
    int nts[3], n = 0;
    for (const char* c = e; *c && n < 3;) {
      nts[n++] = atoi(c);
      while (*c && *c != ',') ++c;
      if (*c == ',') ++c;
    }
    set_march_pref(sh, cls, nts, n);
  }
  ShapeScope shape_scope(&g->shape);   // the levels below take this handle's shape
  lev_dims(g->L0, nx, ny, nz, 1.0);
  if (const char* e = getenv("DSVOF_INNER_MIN")) g->tune.inner_min = atof(e);
  if (const char* e = getenv("DSVOF_INNER_MIN_JAC")) g->tune.inner_min_jac = atof(e);
  if (const char* e = getenv("DSVOF_MG32")) g->tune.mg32 = atoi(e);
  if (const char* e = getenv("DSVOF_NEUMANN")) g->tune.neumann = atoi(e);
  if (const char* e = getenv("DSVOF_ROUND_TEST")) g->tune.round_test = atoi(e);
  if (const char* e = getenv("DSVOF_CONST_Q")) g->tune.const_q = atoi(e);
  if (const char* e = getenv("DSVOF_GRAPHS")) g->tune.graphs = atoi(e);
  if (const char* e = getenv("DSVOF_PHI_DIRECT")) g->tune.phi_direct = atoi(e);
  if (const char* e = getenv("DSVOF_EXTRAP")) g->tune.extrap = atoi(e);
  if (const char* e = getenv("DSVOF_OVERLAP")) g->tune.overlap = atoi(e);
  g->fdm_ok = fdm_supported(P) && P.n < (1LL << 29);
  g->pb_own = g->tune.overlap && prm->pressure_precond == 1 && prm->gas_density == DS_GAS_AMBIENT && !prm->viscous &&
              (prm->precision == DS_PREC_FP64 || (g->tune.mg32 && mg32_supported(g->L0)));
  if (prm->pressure_precond == 1) build_hier(g->H64, nx, ny, nz, prm->h, prm->dt);
  if (prm->precision == DS_PREC_MIXED) {
    if (prm->pressure_precond == 1) build_hier(g->H32, nx, ny, nz, prm->h, prm->dt);
    else lev_dims(g->H32.lev[0], nx, ny, nz, 1.0), g->H32.nlev = 1;
  }
  g->ws_bytes = carve(g, nullptr);
  if (hipHostMalloc((void**)&g->h_scal, SC_COUNT * sizeof(double), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&g->h_status, 4 * sizeof(SolveStatus), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void**)&g->h_grad, GR_COUNT * sizeof(double), hipHostMallocDefault) != hipSuccess) {
    if (g->h_scal) (void)hipHostFree(g->h_scal);
    if (g->h_status) (void)hipHostFree(g->h_status);
    delete g;
    return DS_ERR_HIP;
  }
  *out = g;
  return DS_OK;
}

int ds_destroy_grid(ds_grid* g) {
  if (!g) return DS_ERR_ARG;
  drop_graphs(g);
  if (g->cap_stream) (void)hipStreamDestroy(g->cap_stream);
  if (g->s2) (void)hipStreamDestroy(g->s2);
  if (g->ev_fork) (void)hipEventDestroy(g->ev_fork);
  if (g->ev_join) (void)hipEventDestroy(g->ev_join);
  for (int e = 0; e < 2 * ds_grid::NEV; ++e)
    if (g->ev[e]) (void)hipEventDestroy(g->ev[e]);
  if (g->h_scal) (void)hipHostFree(g->h_scal);
  if (g->h_status) (void)hipHostFree(g->h_status);
  if (g->h_grad) (void)hipHostFree(g->h_grad);
  delete g;
  return DS_OK;
}

size_t ds_workspace_bytes(const ds_grid* g) { return g ? g->ws_bytes : 0; }

int ds_set_fields(ds_grid* g, const double* alpha, const double* T, const double* omega, const double* u,
                  const double* v, const double* w, const double* p, void* workspace, size_t workspace_bytes,
                  void* stream) {
  if (!g) return DS_ERR_ARG;
  ShapeScope shape_scope(&g->shape);
  if (!alpha || !T || !omega || !u || !v || !w || !p || !workspace)
    return fail(g, DS_ERR_ARG, "null pointer argument");
  if (workspace_bytes < g->ws_bytes)
    return fail(g, DS_ERR_ARG, "workspace too small: %zu < %zu bytes", workspace_bytes, g->ws_bytes);
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(g, DS_ERR_ARG, "workspace not 256-byte aligned");
  hipStream_t s = S(stream);
  drop_graphs(g);
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
  if (g->pb_own) HIPCHK(g, hipMemsetAsync(g->pb[1].counters, 0, CT_COUNT * sizeof(unsigned), s));
  HIPCHK(g, hipMemsetAsync(g->scal, 0, SC_COUNT * sizeof(double), s));
  HIPCHK(g, hipMemsetAsync(g->mdot, 0, nb, s));
  HIPCHK(g, hipMemsetAsync(g->mraw, 0, nb, s));
  HIPCHK(g, hipMemsetAsync(g->phi, 0, nb, s));
  launch_xi(g->dp, g->xi, s);
  g->corr_ok = false;
  // conservative vapour variable c = rho_G theta omega (gas fraction only); a variable gas takes
  // rho_G from eq. 24 at each cell's T and omega
  if (g->prm.gas_density) launch_gas_from_omega(g->dp, g->T, g->omega, g->alpha, g->rg, g->c, s);
  else launch_c_from_omega(g->dp, g->alpha, g->omega, g->c, s);
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
  ShapeScope shape_scope(&g->shape);
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
  ShapeScope shape_scope(&g->shape);
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
  ShapeScope shape_scope(&g->shape);
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  hipStream_t s = S(stream);
  const DevParams& P = g->dp;
  int st;
  if ((st = evaporation_source(g, s)) != DS_OK) return st;
  launch_predictor(P, g->alpha, g->xi, g->u, g->v, g->w, g->us, g->vs, g->ws, s);
  if (P.viscous) {
    int itv = 0;
    double resv = 0.0;
    st = viscous_solve(g, g->alpha, s, &itv, &resv, P);
    if (st != DS_OK && st != DS_ERR_NOT_CONVERGED) return st;
    g->diag_out.iters_visc = itv;
    g->diag_out.res_visc = resv;
  }
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

int ds_solve_system(ds_grid* g, int which, const double* rhs, double* x, void* stream, int* iters, double* rel_res) {
  if (!g) return DS_ERR_ARG;
  ShapeScope shape_scope(&g->shape);
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  if (!rhs || !x) return fail(g, DS_ERR_ARG, "null pointer argument");
  if (which < DS_SYS_PRESSURE || which > DS_SYS_POTENTIAL) return fail(g, DS_ERR_ARG, "unknown system %d", which);
  hipStream_t s = S(stream);
  const DevParams& P = g->dp;
  // Assemble the operator from the current state, exactly as the step's setup
  // of that system does (the state's alpha in the role of alpha', its
  // velocities for the inletOutlet switches); the setup's right-hand side is
  // then replaced by the caller's.
  int sys = 0;
  double sc = 0.0, tol = g->prm.tol;
  bool own_phi = false;
  switch (which) {
    case DS_SYS_PRESSURE:
      launch_pressure_setup(P, g->alpha, g->mdot, g->u, g->v, g->w, g->qc, g->diag, g->b, s, f32_out(g, 2));
      sys = 2;
      sc = P.dt / (P.h * P.h);
      break;
    case DS_SYS_ENERGY:
      launch_energy_setup(P, g->alpha, g->T, g->mdot, g->u, g->v, g->w, g->qc, g->diag, g->b, s, f32_out(g, 0));
      sys = 0;
      sc = 1.0 / (P.h * P.h);
      break;
    case DS_SYS_SPECIES:
      launch_species_setup(P, g->alpha, g->c, g->mdot, g->u, g->v, g->w, g->qc, g->diag, g->b, nullptr, s,
                           f32_out(g, 1));
      sys = 1;
      sc = (P.rg ? 1.0 : P.rho_G) * P.D / (P.h * P.h);   // a variable gas: the state's rho_G in the cell coefficient
      break;
    default: {   // the liquid-transport potential, with the step's operator arrays
      own_phi = !potential_direct(g) && g->prm.precision == DS_PREC_MIXED && g->prm.pressure_precond == 1 &&
                g->tune.mg32 && mg32_supported(g->L0);
      if (own_phi) launch_div_setup(P, g->u, g->v, g->w, g->phi_ready ? nullptr : g->phi_qc, g->diag, g->b, s);
      else if (potential_direct(g)) launch_div_setup(P, g->u, g->v, g->w, g->qc, g->diag, g->b, s);
      else launch_div_setup(P, g->u, g->v, g->w, g->qc, g->diag, g->b, s, f32_out(g, 2));
      sys = 2;
      sc = P.dt / (P.h * P.h);
      tol = g->prm.tol_phi;
    }
  }
  HIPCHK(g, hipMemcpyAsync(g->b, rhs, g->n * sizeof(double), hipMemcpyDeviceToDevice, s));
  HIPCHK(g, hipGetLastError());
  int it = 0;
  double res = 0.0;
  int st;
  if (which == DS_SYS_POTENTIAL) {
    st = solve_potential(g, x, s, &it, &res, tol, own_phi);
  } else {
    st = solve(g, sys, sc, x, s, &it, &res, tol);
  }
  if (st != DS_OK && st != DS_ERR_NOT_CONVERGED) return st;
  // The residual reported is the true FP64 one of the returned x: the solvers
  // test the recursively updated residual, which drifts from b - A x when the
  // start is far from the solution (by about eps ||b - A x0||).
  Lev<double> L = g->L0;
  L.sc = sc;
  L.qc = own_phi ? g->phi_qc : g->qc;
  L.diag = g->diag;
  pressure_type(g, sys, L);
  if (own_phi && g->tune.const_q) L.qk = 1.0 / P.dt;
  if ((st = init_status(g, sys, tol, g->prm.maxit, s)) != DS_OK) return st;
  launch_resid64(L, g->b, x, g->r, g->status + sys, g->partials, g->counters + CT_SOLVE0, true, s);
  HIPCHK(g, hipGetLastError());
  if ((st = sync_status(g, sys, s)) != DS_OK) return st;
  res = g->h_status[sys].res;
  if (iters) *iters = it;
  if (rel_res) *rel_res = res;
  if (!(res <= tol))
    return fail(g, DS_ERR_NOT_CONVERGED, "system %d: relative residual %.3e after %d iterations (tol %.3e)", which,
                res, it, tol);
  return DS_OK;
}

int ds_evaporation_rate(ds_grid* g, double* kg_per_s, double* mdot_or_null, void* stream) {
  if (!g) return DS_ERR_ARG;
  ShapeScope shape_scope(&g->shape);
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
  ShapeScope shape_scope(&g->shape);
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
  ShapeScope shape_scope(&g->shape);
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
    case DS_FIELD_RHO_G: src = g->rg; break;
    default: return fail(g, DS_ERR_ARG, "unknown internal field %d", which);
  }
  if (count != n) return fail(g, DS_ERR_ARG, "buffer holds %zu values, field has %zu", count, n);
  if (which == DS_FIELD_ADJ) launch_int_to_double(g->adj, dst, g->n, s);
  else if (which == DS_FIELD_RHO_G && !src) launch_fill(dst, g->dp.rho_G, g->n, s);
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
  return ds_time_kernel(g, DS_KERNEL_CG_OPERATOR, reps, avg_us, bytes_per_launch, stream);
}

int ds_time_kernel(ds_grid* g, int which, int reps, double* avg_us, double* bytes_per_launch, void* stream) {
  if (!g || reps < 1 || !avg_us) return DS_ERR_ARG;
  ShapeScope shape_scope(&g->shape);
  if (which != DS_KERNEL_CG_OPERATOR && which != DS_KERNEL_MG_SMOOTH) return fail(g, DS_ERR_ARG, "unknown kernel %d", which);
  if (which == DS_KERNEL_MG_SMOOTH && g->prm.pressure_precond != 1)
    return fail(g, DS_ERR_ARG, "the multigrid smoother needs pressure_precond = 1");
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
  const bool smooth = which == DS_KERNEL_MG_SMOOTH;
  if (g->prm.precision == DS_PREC_MIXED) {
    // the pressure's arrays: its own set where ds_step overlaps it with the energy and species solves
    const PBufs& B = g->pb_own ? g->pb[1] : g->pb[0];
    Lev<float> F;
    lev_dims(F, P.nx, P.ny, P.nz, P.dt / (P.h * P.h));
    F.qc = B.qc32;
    F.diag = B.diag32;
    if (g->prm.pressure_precond == 1) {   // the fine level of the pressure V-cycle
      F.dfly = 1;
      F.dmask = g->dirmask;
    }
    const bool z32 = g->prm.pressure_precond == 1 && g->tune.mg32 && mg32_supported(g->L0);
    if (smooth) {
      us = replay_smooth_kernel<float>(F, g->H32, B.r32, g->H32.x[0], g->H32.t[0], st, reps, s, g->ev[0],
                                       g->ev[1]);
      // r, x, q read and x written (diag too unless formed from q)
      if (bytes_per_launch) *bytes_per_launch = (F.dfly ? 16.0 : 20.0) * (double)g->n;
    } else if (z32) {
      // the pressure solve's operator: FP64 with the FP32 preconditioned residual z
      Lev<double> L = g->L0;
      L.sc = P.dt / (P.h * P.h);
      L.qc = B.qc;
      L.diag = B.diag;
      pressure_type(g, 2, L);
      us = replay_operator_z32(L, B.r32, B.p32, B.p32alt, B.q, st, g->partials, g->counters + CT_MISC, reps, s,
                               g->ev[0], g->ev[1]);
      // z and p (FP32), q_coef read; p (FP32), q written (diag formed from q_coef)
      if (bytes_per_launch) *bytes_per_launch = 28.0 * (double)g->n;
    } else {
      us = replay_operator_kernel<float>(F, g->r32, g->p32, g->p32alt, g->q32, st, g->partials,
                                         g->counters + CT_MISC, reps, s, g->ev[0], g->ev[1]);
      if (bytes_per_launch) *bytes_per_launch = 24.0 * (double)g->n;
    }
  } else {
    const PBufs& B = g->pb_own ? g->pb[1] : g->pb[0];
    Lev<double> L = g->L0;
    L.sc = P.dt / (P.h * P.h);
    L.qc = B.qc;
    L.diag = B.diag;
    if (g->prm.pressure_precond == 1) pressure_type(g, 2, L);
    if (smooth)
      us = replay_smooth_kernel<double>(L, g->H64, B.r, g->H64.x[0], g->H64.t[0], st, reps, s, g->ev[0],
                                        g->ev[1]);
    else
      us = replay_operator_kernel<double>(L, B.r, B.pd, B.p_alt, B.q, st, g->partials, g->counters + CT_MISC,
                                          reps, s, g->ev[0], g->ev[1]);
    if (bytes_per_launch) *bytes_per_launch = (smooth ? 40.0 : 48.0) * (double)g->n - (L.dfly ? 8.0 * (double)g->n : 0.0);
  }
  if (us < 0) return fail(g, DS_ERR_HIP, "event timing failed");
  *avg_us = us;
  return DS_OK;
}

size_t ds_tape_bytes(const ds_grid* g, int nsteps, int ckpt_every) {
  if (!g || nsteps < 1 || ckpt_every < 1) return 0;
  return tape_total_bytes(g, nsteps, std::min(ckpt_every, nsteps));
}

int ds_forward_record(ds_grid* g, int nsteps, int ckpt_every, void* tape, size_t tape_bytes, void* stream) {
  if (!g) return DS_ERR_ARG;
  ShapeScope shape_scope(&g->shape);
  if (!g->bound) return fail(g, DS_ERR_STATE, "ds_set_fields has not been called");
  if (nsteps < 1 || ckpt_every < 1 || !tape) return fail(g, DS_ERR_ARG, "nsteps and ckpt_every must be >= 1, tape non-null");
  if (g->prm.species_form != DS_SPECIES_CONSERVATIVE)
    return fail(g, DS_ERR_ARG, "the adjoint covers the conservative species form only");
  if (g->prm.viscous) return fail(g, DS_ERR_ARG, "the adjoint covers the inviscid step only");
  if (g->prm.gas_density) return fail(g, DS_ERR_ARG, "the adjoint covers the ambient gas density only");
  if (g->prm.advection) return fail(g, DS_ERR_ARG, "the adjoint covers the flux-limited advection only");
  const int C = std::min(ckpt_every, nsteps);
  const size_t need = tape_total_bytes(g, nsteps, C);
  if (tape_bytes < need) return fail(g, DS_ERR_ARG, "tape too small: %zu < %zu bytes", tape_bytes, need);
  if (reinterpret_cast<uintptr_t>(tape) % 256 != 0) return fail(g, DS_ERR_ARG, "tape not 256-byte aligned");
  hipStream_t s = S(stream);
  g->recorded = false;
  g->tape = static_cast<char*>(tape);
  g->tape_bytes = tape_bytes;
  g->tape_steps = nsteps;
  g->tape_ckpt = C;
  RecordingScope record_scope(g);
  carve_tape(g, g->tape);
  if (g->tape_slot_off != tape_adjoint_bytes(g))
    return fail(g, DS_ERR_STATE, "internal: tape layout carves %zu bytes, sized for %zu", g->tape_slot_off,
                tape_adjoint_bytes(g));
  const int nck = tape_nckpt(nsteps, C);
  int st, rc = DS_OK;
  if ((st = save_slot(g, slot_at(g, 0), s)) != DS_OK) return st;
  for (int k = 0; k < nsteps; ++k) {
    st = one_step(g, s);
    if (st == DS_ERR_NOT_CONVERGED) rc = st;
    else if (st != DS_OK) return st;
    if ((k + 1) % C == 0 && k + 1 < nsteps)
      if ((st = save_slot(g, slot_at(g, (k + 1) / C), s)) != DS_OK) return st;
  }
  if ((st = save_slot(g, slot_at(g, nck), s)) != DS_OK) return st;
  HIPCHK(g, hipStreamSynchronize(s));
  g->fuel_mass_final = g->fuel_mass_prev;
  g->diag_final = g->diag_out;
  g->recorded = true;
  if (rc == DS_OK) g->err.clear();
  return rc;
}

int ds_adjoint(ds_grid* g, double dJ_dV, double* grads, double* dalpha0, double* dT0, double* domega0, double* du0,
               double* dv0, double* dw0, void* stream) {
  if (!g || !grads) return DS_ERR_ARG;
  ShapeScope shape_scope(&g->shape);
  if (!g->recorded) return fail(g, DS_ERR_STATE, "ds_forward_record has not been called");
  if (!std::isfinite(dJ_dV)) return fail(g, DS_ERR_ARG, "dJ_dV is not finite");
  hipStream_t s = S(stream);
  RecordingScope record_scope(g);
  const DevParams& P = g->dp;
  const int N = g->tape_steps, C = g->tape_ckpt, nck = tape_nckpt(N, C);
  int st, rc = DS_OK;
  for (int q = 0; q < 4; ++q) g->adj_iters[q] = 0;
  // adjoint of V_N = h^3 sum(alpha^N)
  launch_fill(g->A_al, P.h * P.h * P.h * dJ_dV, g->n, s);
  launch_fill(g->A_c, 0.0, g->n, s);
  launch_fill(g->A_om, 0.0, g->n, s);
  launch_fill(g->A_T, 0.0, g->n, s);
  launch_fill(g->A_U[0], 0.0, g->nu, s);
  launch_fill(g->A_U[1], 0.0, g->nv, s);
  launch_fill(g->A_U[2], 0.0, g->nw, s);
  launch_fill(g->grad, 0.0, GR_COUNT, s);
  HIPCHK(g, hipGetLastError());
  for (int sg = nck - 1; sg >= 0; --sg) {
    const int n0 = sg * C, n1 = std::min(N, n0 + C);
    // recompute the segment's states from its checkpoint (segment slots q = 0.. hold steps n0+1+q)
    if (n1 - n0 > 1) {
      if ((st = load_slot(g, slot_at(g, sg), s)) != DS_OK) return st;
      for (int k = n0; k < n1 - 1; ++k) {
        st = one_step(g, s);
        if (st != DS_OK && st != DS_ERR_NOT_CONVERGED) return st;
        if ((st = save_slot(g, slot_at(g, nck + 1 + (k - n0)), s)) != DS_OK) return st;
      }
    }
    for (int n = n1 - 1; n >= n0; --n) {
      const Slot cur = n == n0 ? slot_at(g, sg) : slot_at(g, nck + 1 + (n - n0 - 1));
      const Slot nxt = n + 1 == n1 ? (n1 == N ? slot_at(g, nck) : slot_at(g, sg + 1)) : slot_at(g, nck + 1 + (n - n0));
      if ((st = reverse_step(g, cur, nxt, s, &rc)) != DS_OK) return st;
    }
  }
  const Slot s0 = slot_at(g, 0);
  launch_adj_init_c(P, s0.alpha, s0.omega, g->A_c, g->A_al, g->A_om, g->partials, g->counters + CT_ADJ, g->grad, s);
  HIPCHK(g, hipGetLastError());
  HIPCHK(g, hipMemcpyAsync(g->h_grad, g->grad, GR_COUNT * sizeof(double), hipMemcpyDeviceToHost, s));
  const size_t nb = g->n * sizeof(double);
  if (dalpha0) HIPCHK(g, hipMemcpyAsync(dalpha0, g->A_al, nb, hipMemcpyDeviceToDevice, s));
  if (dT0) HIPCHK(g, hipMemcpyAsync(dT0, g->A_T, nb, hipMemcpyDeviceToDevice, s));
  if (domega0) HIPCHK(g, hipMemcpyAsync(domega0, g->A_om, nb, hipMemcpyDeviceToDevice, s));
  if (du0) HIPCHK(g, hipMemcpyAsync(du0, g->A_U[0], g->nu * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (dv0) HIPCHK(g, hipMemcpyAsync(dv0, g->A_U[1], g->nv * sizeof(double), hipMemcpyDeviceToDevice, s));
  if (dw0) HIPCHK(g, hipMemcpyAsync(dw0, g->A_U[2], g->nw * sizeof(double), hipMemcpyDeviceToDevice, s));
  // the handle continues from the final state
  if ((st = load_slot(g, slot_at(g, nck), s)) != DS_OK) return st;
  HIPCHK(g, hipStreamSynchronize(s));
  g->fuel_mass_prev = g->fuel_mass_final;
  g->diag_out = g->diag_final;
  grads[0] = g->h_grad[GR_D];
  grads[1] = g->h_grad[GR_DH];
  grads[2] = g->h_grad[GR_TAMB] + g->h_grad[GR_RHOG] * host_drhoG_dT(g->prm, P.rho_G);
  if (!std::isfinite(grads[0]) || !std::isfinite(grads[1]) || !std::isfinite(grads[2]))
    return fail(g, DS_ERR_NONFINITE, "non-finite gradient");
  if (rc != DS_OK) return fail(g, rc, "an adjoint linear solve reached maxit");
  g->err.clear();
  return DS_OK;
}

int ds_get_adjoint_iterations(const ds_grid* g, int* iters4) {
  if (!g || !iters4) return DS_ERR_ARG;
  for (int q = 0; q < 4; ++q) iters4[q] = g->adj_iters[q];
  return DS_OK;
}

int ds_get_diagnostics(const ds_grid* g, ds_diagnostics* out) {
  if (!g || !out) return DS_ERR_ARG;
  *out = g->diag_out;
  return DS_OK;
}

const char* ds_last_error(const ds_grid* g) { return g ? g->err.c_str() : dsv_noalloc_last_error(); }

}  // extern "C"
