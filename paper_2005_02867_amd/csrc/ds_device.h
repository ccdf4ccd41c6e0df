// Device-side helpers shared by the dsvof kernels: grid indexing, the
// XCD-aware block-to-range mapping, deterministic FP64 block reductions and
// the per-launch parameter block.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dsv {

constexpr double R_GAS = 8.314462618;
constexpr int BLOCK = 256;          // 4 wavefronts of 64
constexpr int NXCD = 8;             // MI355X: 8 XCDs, blocks are dealt round-robin
constexpr int MAX_BLOCKS = 2048;    // streaming grids: 256 CUs x 8 blocks
constexpr int MAX_RED = 8;          // values per block partial

enum BoxKind { WALL = 0, INLET = 1, OPEN = 2, FARFIELD = 3 };

// Tiles of the marching stencil kernels: MZ z (one wavefront) by MY y rows,
// marching along x over chunks of xlen planes; nzb x nyb tiles per chunk.
constexpr int MZ = 64, MY = 4;
struct MarchGeom {
  int nzb, nyb, xlen;
  long long tiles;
};

// Parameters passed by value to every kernel.
struct DevParams {
  int nx, ny, nz, smax;
  long long n;                      // cells
  double h, dt, p, T_amb, rho_L, cp_L, k_L, cp_G, k_G, D, dh, M_v, M_G;
  double g[3], x0[3];
  double xi0, Df, r_fib, w_in;
  double Tc, Pc, om, Tc_G, Pc_G, om_G, kij, T_ref, p_ref;
  double eps, eps_gas, theta_min, rho_G;
  int kind[6];                      // box face kinds, index axis*2 + side
  int eq_model, solve_energy, evaporation;
  int species_form;                 // 0 conservative, 1 literal (saturated liquid, central gradient at adj)
  int viscous;                      // 1: implicit viscous momentum (mu_L, mu_G mixed by eq. 31)
  double mu_L, mu_G;
  // variable-density gas: the per-cell rho_G a stage reads (nullptr: the
  // ambient constant rho_G everywhere)
  const double* rg;
};

// Status of one iterative solve, updated on the device.
struct SolveStatus {
  double bnorm;   // ||b||_2
  double rz;      // <r, z>
  double alpha;   // CG step
  double beta;    // CG direction update
  double res;     // ||r||/||b||
  double tol;
  double bb, rr;
  int it, done, maxit, zero;   // done: 0 running, 1 converged, 2 hit maxit
};

__device__ __forceinline__ long long cidx(const DevParams& P, int i, int j, int k) {
  return ((long long)i * P.ny + j) * P.nz + k;
}
__device__ __forceinline__ long long uidx(const DevParams& P, int i, int j, int k) {
  return ((long long)i * P.ny + j) * P.nz + k;
}
__device__ __forceinline__ long long vidx(const DevParams& P, int i, int j, int k) {
  return ((long long)i * (P.ny + 1) + j) * P.nz + k;
}
__device__ __forceinline__ long long widx(const DevParams& P, int i, int j, int k) {
  return ((long long)i * P.ny + j) * (P.nz + 1) + k;
}

// Cell (i, j, k) of flat index c.  Grids hold fewer than 2^31 cells (checked
// at creation), so 32-bit unsigned division is exact and much cheaper than
// the 64-bit form.
__device__ __forceinline__ void decode(const DevParams& P, long long c, int& i, int& j, int& k) {
  const unsigned cu = (unsigned)c, nz = (unsigned)P.nz, ny = (unsigned)P.ny;
  const unsigned t = cu / nz;
  k = (int)(cu - t * nz);
  j = (int)(t % ny);
  i = (int)(t / ny);
}

// (i, j, k) of flat index e in an array of extents (., fy, fz) (face arrays;
// fewer than 2^31 entries, so 32-bit unsigned division is exact).
__device__ __forceinline__ void decode3(long long e, int fy, int fz, int& i, int& j, int& k) {
  const unsigned eu = (unsigned)e, uz = (unsigned)fz, uy = (unsigned)fy;
  const unsigned t = eu / uz;
  k = (int)(eu - t * uz);
  j = (int)(t % uy);
  i = (int)(t / uy);
}

// Contiguous range of items handled by this block.  Blocks are dealt to the
// 8 XCDs round-robin; logical block numbers are permuted so that each XCD
// streams one contiguous eighth of the array (stencil neighbours then hit
// the same L2).  gridDim.x must be a multiple of NXCD.
__device__ __forceinline__ void block_range(long long n, long long& begin, long long& end) {
  const int nb = gridDim.x;
  const int per = nb / NXCD;
  const int logical = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  long long chunk = (n + nb - 1) / nb;
  chunk = (chunk + BLOCK - 1) / BLOCK * BLOCK;
  begin = (long long)logical * chunk;
  end = begin + chunk;
  if (end > n) end = n;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

enum RedOp { RSUM = 0, RMIN = 1, RMAX = 2 };

// Reduce NV values over the block (fixed order) and store them as this
// block's partials.  Returns true in every thread of the last block to
// finish (which may then combine the partials of all blocks).
//
// Publication without an L2 writeback: the partials are stored as
// device-scope atomics, which on the multi-XCD part write through the XCD's
// L2 to the device coherence point; thread 0 waits for those stores to
// complete (s_waitcnt) before it bumps the counter, and the last block reads
// the partials with device-scope atomic loads, which fetch from that point.
// A device-scope release fence would instead write back every dirty line of
// the L2 (the kernel's streamed outputs), which costs tens of microseconds per
// block.  The last block reads nothing else that this launch wrote; the
// outputs reach later kernels through the launch boundary.
template <int NV, int NT = BLOCK>
__device__ bool block_reduce_publish(double (&v)[NV], const int (&ops)[NV], double* partials,
                                     unsigned* counter) {
  __shared__ double sh[NT / 64][NV];
  __shared__ bool last;
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double x = ops[q] == RSUM ? wave_sum(v[q]) : (ops[q] == RMIN ? wave_min(v[q]) : wave_max(v[q]));
    if (lane == 0) sh[wid][q] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      double x = sh[0][q];
      for (int w = 1; w < NT / 64; ++w)
        x = ops[q] == RSUM ? x + sh[w][q] : (ops[q] == RMIN ? fmin(x, sh[w][q]) : fmax(x, sh[w][q]));
      __hip_atomic_store(&partials[(size_t)blockIdx.x * NV + q], x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __builtin_amdgcn_s_waitcnt(0);   // the partial stores have completed
    unsigned prev = atomicAdd(counter, 1u);
    last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  return last;
}

constexpr int pow2_floor(int n) { return n <= 1 ? 1 : 2 * pow2_floor(n / 2); }

// In the last block: combine all partials (fixed order), result in out[q]
// (valid in every thread).  Resets the counter.
template <int NV, int NT = BLOCK>
__device__ void block_combine(const int (&ops)[NV], const double* partials, unsigned* counter,
                              double (&out)[NV]) {
  __shared__ double sh[NT][NV];
  const int nb = gridDim.x;
#pragma unroll
  for (int q = 0; q < NV; ++q) {
    double x = ops[q] == RSUM ? 0.0 : (ops[q] == RMIN ? __builtin_inf() : -__builtin_inf());
    for (int b = threadIdx.x; b < nb; b += NT) {
      double y = __hip_atomic_load(&partials[(size_t)b * NV + q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      x = ops[q] == RSUM ? x + y : (ops[q] == RMIN ? fmin(x, y) : fmax(x, y));
    }
    sh[threadIdx.x][q] = x;
  }
  __syncthreads();
  // tree over the largest power of two P2 <= NT; the threads past P2 (NT =
  // 384: 128 of them) are folded in first
  constexpr int P2 = pow2_floor(NT);
  if (P2 < NT) {
    if (threadIdx.x < NT - P2) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        double a = sh[threadIdx.x][q], b = sh[threadIdx.x + P2][q];
        sh[threadIdx.x][q] = ops[q] == RSUM ? a + b : (ops[q] == RMIN ? fmin(a, b) : fmax(a, b));
      }
    }
    __syncthreads();
  }
  for (int s = P2 / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        double a = sh[threadIdx.x][q], b = sh[threadIdx.x + s][q];
        sh[threadIdx.x][q] = ops[q] == RSUM ? a + b : (ops[q] == RMIN ? fmin(a, b) : fmax(a, b));
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < NV; ++q) out[q] = sh[0][q];
  if (threadIdx.x == 0) atomicExch(counter, 0u);
}

// Gas density of cell c: the stage's field (variable gas) or the constant.
__device__ __forceinline__ double rho_gas(const DevParams& P, long long c) { return P.rg ? P.rg[c] : P.rho_G; }

// Mixing rule of the fluid properties (eq. 31) on alpha clamped to [0, 1].
__device__ __forceinline__ double clamp01(double a) { return fmin(fmax(a, 0.0), 1.0); }
__device__ __forceinline__ double mix(double ab, double liq, double gas) {
  return ab * liq + (1.0 - ab) * gas;
}

// Does the scalar (T, omega) take its ambient value on this boundary face?
// Open faces switch on the sign of the face velocity ("inletOutlet").
__device__ __forceinline__ bool scalar_dirichlet(int kind, double uface, int side) {
  if (kind == WALL) return false;
  if (kind == INLET || kind == FARFIELD) return true;
  return side == 0 ? (uface > 0.0) : (uface < 0.0);
}
__host__ __device__ __forceinline__ bool pressure_dirichlet(int kind) { return kind == OPEN || kind == FARFIELD; }

}  // namespace dsv
