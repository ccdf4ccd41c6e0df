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
  SC_COUNT
};
// Reduction counters (one per reduction site).
enum Counter { CT_IFACE = 0, CT_ADV, CT_SPEC, CT_DIAG, CT_SOLVE0, CT_SOLVE1, CT_SOLVE2, CT_MISC, CT_COUNT };

int grid_blocks(long long n);   // streaming grid size (multiple of 8)

// ---- step kernels (k_step.hip)
void launch_xi(const DevParams& P, double* xi, hipStream_t s);
void launch_interface(const DevParams& P, const double* alpha, const double* T, const double* omega,
                      const double* u, const double* v, const double* w, double* mraw, int* adj,
                      double* partials, unsigned* counter, double* scal, hipStream_t s);
void launch_source(const DevParams& P, const double* alpha, const double* mraw, const double* scal,
                   double* mdot, double* a1, hipStream_t s);
void launch_advect(const DevParams& P, const double* a1, const double* omega, const double* T,
                   const double* c, const double* u, const double* v, const double* w, const double* phi,
                   double* a_new, double* c_new, double* T_new, double* partials, unsigned* counter, double* scal,
                   hipStream_t s);
void launch_div_setup(const DevParams& P, const double* u, const double* v, const double* w, double* qc,
                      double* diag, double* b, hipStream_t s);
void launch_energy_setup(const DevParams& P, const double* a_new, const double* T_prime,
                         const double* mdot, const double* u, const double* v, const double* w,
                         double* qc, double* diag, double* b, hipStream_t s);
void launch_species_setup(const DevParams& P, const double* a_new, const double* c_prime,
                          const double* mdot, const double* u, const double* v, const double* w,
                          double* qc, double* diag, double* b, double* om0, hipStream_t s);
void launch_species_update(const DevParams& P, const double* a_new, const double* c_prime,
                           const double* mdot, const double* om, const double* u, const double* v,
                           const double* w, double* c, double* omega, double* partials,
                           unsigned* counter, double* scal, hipStream_t s);
void launch_predictor(const DevParams& P, const double* a_new, const double* xi, const double* u,
                      const double* v, const double* w, double* us, double* vs, double* ws,
                      hipStream_t s);
void launch_pressure_setup(const DevParams& P, const double* a_new, const double* mdot,
                           const double* us, const double* vs, const double* ws, double* qc,
                           double* diag, double* b, hipStream_t s);
void launch_project(const DevParams& P, const double* a_new, const double* p, const double* us,
                    const double* vs, const double* ws, double* u, double* v, double* w,
                    hipStream_t s);
void launch_diagnostics(const DevParams& P, const double* alpha, const double* c, const double* T,
                        const double* p, const double* mdot, double* partials, unsigned* counter,
                        double* scal, hipStream_t s);
void launch_c_from_omega(const DevParams& P, const double* alpha, const double* omega, double* c, hipStream_t s);
void launch_fill(double* x, double v, long long n, hipStream_t s);
void launch_int_to_double(const int* src, double* dst, long long n, hipStream_t s);

}  // namespace dsv
