// Host-side launch wrappers of the dsvof kernels (one stream, async).
#pragma once
#include <hip/hip_runtime.h>

#include "ds_device.h"

namespace dsv {

// Device scalar slots (doubles) shared by the step kernels.
enum Scalar {
  SC_K = 0, SC_S1, SC_S2, SC_NINT,
  SC_BL, SC_BV_ADV, SC_BV_DIFF,
  SC_VOL, SC_FUEL, SC_MDOT, SC_AMIN, SC_AMAX, SC_NONFINITE,
  SC_ABSMAX,
  SC_COUNT
};
// Reduction counters (one per reduction site).
enum Counter { CT_IFACE = 0, CT_ADV, CT_SPEC, CT_DIAG, CT_SOLVE0, CT_SOLVE1, CT_SOLVE2, CT_MISC, CT_ADJ, CT_COUNT };
// Device gradient accumulators of the differentiation form.
enum Grad { GR_D = 0, GR_DH, GR_TAMB, GR_RHOG, GR_S1B, GR_S2B, GR_COUNT };

int grid_blocks(long long n);   // streaming grid size (multiple of 8)
MarchGeom march_geom(const DevParams& P, int& blocks);   // tiles and grid of the marching kernels

// FP32 copies of an assembled operator for the precision form, written by the
// setup kernels next to the FP64 ones (q null: none).  d: the FP32 diagonal,
// (float) of the FP64 one, or with mg the multigrid's own formula on the FP32
// q values (what k_mg_diag computes; sc: the FP32 level's scale, widened).
struct F32Out {
  float* q = nullptr;
  float* d = nullptr;
  int mg = 0;
  double sc = 0.0;
};

// ---- step kernels (k_step.hip)
void launch_xi(const DevParams& P, double* xi, hipStream_t s);
// Interface cells in two passes (a scan writing per-block lists of interface
// cells into band/band_count, then the march and flux on those cells only).
void launch_interface(const DevParams& P, const double* alpha, const double* T, const double* omega,
                      const double* u, const double* v, const double* w, double* mraw, int* adj, int* band,
                      int* band_count, double* partials, unsigned* counter, double* scal, hipStream_t s);
long long interface_band_capacity(long long n);   // ints needed for `band`
// Literal species form: omega = omega_sat(T), c = rho_G theta omega in every
// cell with alpha > eps_gas; other cells untouched.  Uses band and
// band_count (as launch_interface) for the list of liquid cells.
void launch_liquid_saturation(const DevParams& P, const double* alpha, const double* T, double* omega, double* c,
                              int* band, int* band_count, hipStream_t s);
// band_count: 2 * MAX_BLOCKS + 1 ints (per-block counts, then their offsets).
void launch_source(const DevParams& P, const double* alpha, const double* mraw, const double* scal,
                   double* mdot, double* a1, hipStream_t s);
void launch_advect(const DevParams& P, const double* a1, const double* omega, const double* T,
                   const double* c, const double* u, const double* v, const double* w, const double* phi,
                   double* a_new, double* c_new, double* T_new, double* partials, unsigned* counter, double* scal,
                   hipStream_t s, const double* Fx = nullptr, const double* Fy = nullptr,
                   const double* Fz = nullptr);   // Fx..Fz: given liquid fluxes (geometric advection)
void launch_div_setup(const DevParams& P, const double* u, const double* v, const double* w, double* qc,
                      double* diag, double* b, hipStream_t s, F32Out fo = {});
void launch_energy_setup(const DevParams& P, const double* a_new, const double* T_prime,
                         const double* mdot, const double* u, const double* v, const double* w,
                         double* qc, double* diag, double* b, hipStream_t s, F32Out fo = {});
void launch_species_setup(const DevParams& P, const double* a_new, const double* c_prime,
                          const double* mdot, const double* u, const double* v, const double* w,
                          double* qc, double* diag, double* b, double* om0, hipStream_t s, F32Out fo = {},
                          const double* corr = nullptr);
void launch_species_update(const DevParams& P, const double* a_new, const double* c_prime,
                           const double* mdot, const double* om, const double* u, const double* v,
                           const double* w, double* c, double* omega, double* partials,
                           unsigned* counter, double* scal, hipStream_t s, double* corr = nullptr);
void launch_predictor(const DevParams& P, const double* a_new, const double* xi, const double* u,
                      const double* v, const double* w, double* us, double* vs, double* ws,
                      hipStream_t s);
void launch_pressure_setup(const DevParams& P, const double* a_new, const double* mdot,
                           const double* us, const double* vs, const double* ws, double* qc,
                           double* diag, double* b, hipStream_t s, F32Out fo = {},
                           const double* scomp = nullptr);   // scomp: variable gas's compressibility term
void launch_project(const DevParams& P, const double* a_new, const double* p, const double* us,
                    const double* vs, const double* ws, double* u, double* v, double* w,
                    hipStream_t s);
// The projection and, in the same pass, the diagnostics of launch_diagnostics
// over alpha = a_new (the state after the step), c, T, p and mdot.
void launch_project_diagnostics(const DevParams& P, const double* a_new, const double* p, const double* us,
                                const double* vs, const double* ws, double* u, double* v, double* w,
                                const double* c, const double* T, const double* mdot, double* partials,
                                unsigned* counter, double* scal, hipStream_t s);
void launch_diagnostics(const DevParams& P, const double* alpha, const double* c, const double* T,
                        const double* p, const double* mdot, double* partials, unsigned* counter,
                        double* scal, hipStream_t s);
void launch_c_from_omega(const DevParams& P, const double* alpha, const double* omega, double* c, hipStream_t s);
// geometric interface advection (k_geo.hip): planes of the surface cells, liquid fluxes per face
void launch_geo_fluxes(const DevParams& P, const double* a1, const double* u, const double* v, const double* w,
                       const double* phi, double* const (&planes)[4], double* Fx, double* Fy, double* Fz,
                       hipStream_t s);
// variable-density gas (k_gas.hip)
void launch_gas_from_omega(const DevParams& P, const double* T, const double* omega, const double* alpha, double* rg,
                           double* c, hipStream_t s);
void launch_gas_partial(const DevParams& P, const double* omega, const double* rg, double* q, hipStream_t s);
void launch_gas_invert(const DevParams& P, const double* T, const double* c, const double* alpha, double* rg,
                       hipStream_t s);
void launch_gas_end(const DevParams& P, const double* T, const double* c, const double* alpha, const double* rg_adv,
                    double* omega, double* rg, double* scomp, hipStream_t s);
void launch_fill(double* x, double v, long long n, hipStream_t s);
// max |x| (non-finite entries give +inf) -> *out; x *= a
void launch_absmax(const double* x, long long n, double* partials, unsigned* counter, double* out, hipStream_t s);
void launch_scale(double* x, double a, long long n, hipStream_t s);

// ---- direct solve of the liquid-transport potential (k_fdm.hip)
// The potential's matrix c_op (A_x + A_y + A_z) (unit second differences with
// the pressure's box faces) is diagonalised by DCT-II / DST-II bases.  Needs
// each lateral axis with equal faces (walls or phi = 0), phi = 0 at z+, and
// extents 4^a 2^b 3^c (2 nz for z with a no-flux z- face) of at most 1024.
bool fdm_supported(const DevParams& P);
// x = A^-1 b in five passes (t: scratch cell array); -1 if not supported.
int launch_fdm_solve(const DevParams& P, double c_op, const double* b, double* x, double* t, hipStream_t s);

// ---- implicit viscous momentum (k_visc.hip)
// Work vectors of the viscous solve, each over the concatenated faces
// [u | v | w] (visc_faces entries).
struct ViscVecs {
  double *x, *b, *d, *r, *p, *q;
};
long long visc_faces(const DevParams& P);
// x = (u*, v*, w*), right-hand side and diagonal, r = b - A x, p = r/d and
// the status (bnorm, rz, residual, done) of the solve.
void launch_visc_start(const DevParams& P, const double* a_new, const double* us, const double* vs, const double* ws,
                       const double* u, const double* v, const double* w, const ViscVecs& X, SolveStatus* st,
                       double* partials, unsigned* counter, hipStream_t s);
// One Jacobi-PCG iteration (three launches; each returns at once after convergence).
void launch_visc_iteration(const DevParams& P, const double* a_new, const ViscVecs& X, SolveStatus* st,
                           double* partials, unsigned* counter, hipStream_t s);
// The interior faces of x back into u*, v*, w*.
void launch_visc_store(const DevParams& P, const ViscVecs& X, double* us, double* vs, double* ws, hipStream_t s);

// ---- adjoint kernels (k_adjoint.hip), in the order of the reverse step
void launch_adj_project(const DevParams& P, const double* a_new, const double* p, double* const AU[3], double* b,
                        double* A_ab, double* partials, unsigned* counter, double* grad, hipStream_t s);
void launch_adj_pressure(const DevParams& P, const double* a_new, const double* p, const double* lam,
                         const double* mdot, double* A_ab, double* A_md, double* partials, unsigned* counter,
                         double* grad, hipStream_t s);
void launch_adj_predictor(const DevParams& P, const double* a_new, const double* xi, double* const AU[3],
                          double* const AUs[3], double* const Q[6], const double* lam, const double* u,
                          const double* v, const double* w, double* A_ab, double* partials, unsigned* counter,
                          double* grad, hipStream_t s);
void launch_adj_species_rhs(const DevParams& P, const double* a_new, const double* omt, const double* A_om,
                            const double* A_c, double* b, double* A_ab, double* partials, unsigned* counter,
                            double* grad, hipStream_t s);
void launch_adj_species(const DevParams& P, const double* a_new, const double* omt, const double* lam,
                        const double* u, const double* v, const double* w, double* A_ab, double* A_cp, double* A_md,
                        double* partials, unsigned* counter, double* grad, hipStream_t s);
void launch_adj_energy(const DevParams& P, const double* a_new, const double* Tp, const double* Tn, const double* lam,
                       const double* mdot, const double* u, const double* v, const double* w, double* A_ab,
                       double* A_Tp, double* A_md, double* partials, unsigned* counter, double* grad, hipStream_t s);
void launch_adj_advect(const DevParams& P, const double* a1, const double* omega, const double* T, const double* u,
                       const double* v, const double* w, const double* phi, const double* a_new, const double* A_al,
                       const double* A_ab, const double* A_cp, const double* A_Tp, double* const AU[3],
                       double* const AUl[3], double* A_a1, double* A_om, double* A_T, double* A_c, double* partials,
                       unsigned* counter, double* grad, hipStream_t s);
void launch_adj_phi_rhs(const DevParams& P, double* const AUl[3], double* b, hipStream_t s);
void launch_adj_phi_faces(const DevParams& P, double* const AUl[3], const double* lam, double* const AU[3],
                          hipStream_t s);
void launch_adj_source(const DevParams& P, const double* alpha, const double* mraw, const double* A_a1, double* A_md,
                       double* A_al, const double* scal, double* partials, unsigned* counter, double* grad,
                       hipStream_t s);
// Per-cell records of the adjoint interface stage (tape arrays): see k_adjoint.hip.
struct IfaceRecords {
  double* gb[3];    // to alpha of the neighbours -+q
  double* om;       // to omega of adj
  double* f[3];     // to each of adj's two q faces
  double* gsf[3];   // per adj cell: sum of its band cells' f[q]
  double* hit;      // 1 where a band cell's adj is this cell
  int* list;        // the cells marked in hit, once each (in no particular order)
  unsigned* rmax;   // largest march distance (cells, Chebyshev)
  unsigned* nlist;  // length of list
};
void launch_adj_interface(const DevParams& P, const double* alpha, const double* T, const double* omega,
                          const double* u, const double* v, const double* w, const double* mraw, const int* adj,
                          const double* A_md, const double* scal, double* A_al, double* A_T, double* A_om,
                          double* const AU[3], const IfaceRecords& R, double* partials, unsigned* counter,
                          double* grad, hipStream_t s);
void launch_adj_init_c(const DevParams& P, const double* alpha, const double* omega, const double* A_c, double* A_al,
                       double* A_om, double* partials, unsigned* counter, double* grad, hipStream_t s);
void launch_int_to_double(const int* src, double* dst, long long n, hipStream_t s);

}  // namespace dsv
