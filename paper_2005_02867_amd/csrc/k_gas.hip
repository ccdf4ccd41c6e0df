// Variable-density gas (gas_density = 1): per-cell eq. 24, the state's
// (omega, rho_G) from (T, c), and eq. 7's compressibility term
// (1 - alpha)(1/rho_G) D rho_G/Dt over the step.  Streaming kernels, one
// thread per cell (the Peng-Robinson root makes them ALU-bound).
#include <hip/hip_runtime.h>

#include "ds_device.h"
#include "ds_gas.h"
#include "ds_kernels.h"

namespace dsv {

namespace {

__device__ __forceinline__ double gas_theta(const DevParams& P, double a) {
  return fmax(1.0 - clamp01(a), P.theta_min);
}

// rho_G = eq. 24 at (T, omega), c = rho_G theta omega (a state from omega).
__global__ void __launch_bounds__(BLOCK) k_gas_from_omega(DevParams P, const double* __restrict__ T, const double* __restrict__ omega,
                                 const double* __restrict__ alpha, double* __restrict__ rg, double* __restrict__ c) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    const double r = gas_rho<double>(P, T[e], omega[e]);
    rg[e] = r;
    c[e] = r * gas_theta(P, alpha[e]) * omega[e];
  }
}

// q = rho_G omega: the vapour mass per unit gas volume the advection carries.
__global__ void __launch_bounds__(BLOCK) k_gas_partial(DevParams P, const double* __restrict__ omega, const double* __restrict__ rg,
                              double* __restrict__ q) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) q[e] = rg[e] * omega[e];
}

// rho_G of the advected state (T', c', alpha').
__global__ void __launch_bounds__(BLOCK) k_gas_invert(DevParams P, const double* __restrict__ T, const double* __restrict__ c,
                             const double* __restrict__ alpha, double* __restrict__ rg) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    double om, r;
    gas_invert(P, T[e], c[e] / gas_theta(P, alpha[e]), om, r);
    rg[e] = r;
  }
}

// End of the step: (omega, rho_G) from (T^{n+1}, c^{n+1}, alpha') and the
// compressibility term (1 - alpha') log1p((rho^{n+1} - rho')/rho')/dt.
__global__ void __launch_bounds__(BLOCK) k_gas_end(DevParams P, const double* __restrict__ T, const double* __restrict__ c,
                          const double* __restrict__ alpha, const double* __restrict__ rg_adv,
                          double* __restrict__ omega, double* __restrict__ rg, double* __restrict__ scomp) {
  long long b0, b1;
  block_range(P.n, b0, b1);
  for (long long e = b0 + threadIdx.x; e < b1; e += BLOCK) {
    const double a = alpha[e];
    double om, r;
    gas_invert(P, T[e], c[e] / gas_theta(P, a), om, r);
    omega[e] = om;
    rg[e] = r;
    const double ra = rg_adv[e];
    scomp[e] = (1.0 - clamp01(a)) * log1p((r - ra) / ra) / P.dt;
  }
}

}  // namespace

void launch_gas_from_omega(const DevParams& P, const double* T, const double* omega, const double* alpha, double* rg,
                           double* c, hipStream_t s) {
  k_gas_from_omega<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, T, omega, alpha, rg, c);
}
void launch_gas_partial(const DevParams& P, const double* omega, const double* rg, double* q, hipStream_t s) {
  k_gas_partial<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, omega, rg, q);
}
void launch_gas_invert(const DevParams& P, const double* T, const double* c, const double* alpha, double* rg,
                       hipStream_t s) {
  k_gas_invert<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, T, c, alpha, rg);
}
void launch_gas_end(const DevParams& P, const double* T, const double* c, const double* alpha, const double* rg_adv,
                    double* omega, double* rg, double* scomp, hipStream_t s) {
  k_gas_end<<<grid_blocks(P.n), BLOCK, 0, s>>>(P, T, c, alpha, rg_adv, omega, rg, scomp);
}

}  // namespace dsv
