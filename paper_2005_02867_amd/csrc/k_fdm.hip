// Direct solve of the liquid-transport potential's system by fast
// diagonalisation.
//
// The potential of the divergent part of the face velocities solves
// D G phi = D u (interface advection, eq. 3, with the divergence-free part of
// u) with the pressure's boundary kinds and a constant face coefficient c_op
// (= (dt/h^2)(1/dt)).  Its matrix is c_op (A_x + A_y + A_z), a sum of
// one-dimensional second differences with unit coefficients, each of which
// has a closed-form eigenbasis:
//   both faces without flux (walls):       cos(pi k (n+1/2)/N), eigenvalue 4 sin^2(pi k/(2N))
//   both faces at phi = 0 (open, far field): sin(pi (k+1)(n+1/2)/N), 4 sin^2(pi (k+1)/(2N))
//   no flux at z-, phi = 0 at z+ (forced inlet): the second basis on the line
//   mirrored about the z- face (length 2N), whose symmetric modes are the
//   line's eigenvectors.
// Projections onto the first basis are DCT-II coefficients, onto the second
// DST-II coefficients; both are computed here through complex FFTs of the
// reordered line (two real lines packed into one complex line), so
//   phi = T^-1 [ (T b) / (c_op (l_x + l_y + l_z)) ],   T = T_z T_y T_x,
// in five passes over the grid: forward along x and along y, the whole z
// solve (forward, division by the eigenvalue sum, inverse) on contiguous
// lines, inverse along y and along x.  The result is exact up to rounding
// (no iteration).  Every pass streams the grid once (read and write), and
// the FFTs run in LDS (Stockham, radices 4, 2 and 3).
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ds_device.h"
#include "ds_kernels.h"

namespace dsv {

namespace {

constexpr int FDM_NT = 256;          // threads per workgroup
constexpr int FDM_LAT_LINES = 16;    // real lines per workgroup of a lateral pass (16 consecutive z)
constexpr int FDM_MAXLEN = 1024;     // longest transform

struct Cx {
  double re, im;
};

struct FftPlan {
  int n;        // transform length
  int nr;       // radix passes
  int r[16];    // radices in pass order
};

// n = 4^a 2^b 3^c (b <= 1): radix-4 passes, then a radix-2 pass, then radix-3 passes.
bool make_plan(int n, FftPlan& pl) {
  if (n < 1 || n > FDM_MAXLEN) return false;
  pl.n = n;
  pl.nr = 0;
  int m = n;
  while (m % 4 == 0 && pl.nr < 16) pl.r[pl.nr++] = 4, m /= 4;
  if (m % 2 == 0 && pl.nr < 16) pl.r[pl.nr++] = 2, m /= 2;
  while (m % 3 == 0 && pl.nr < 16) pl.r[pl.nr++] = 3, m /= 3;
  return m == 1;
}

__device__ __forceinline__ Cx cmul(Cx a, Cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ Cx cadd(Cx a, Cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ Cx csub(Cx a, Cx b) { return {a.re - b.re, a.im - b.im}; }
// s i a (s = +-1)
__device__ __forceinline__ Cx cmuli(Cx a, double s) { return {-s * a.im, s * a.re}; }

// e^{i pi x}
__device__ __forceinline__ Cx cispi(double x) {
  Cx w;
  sincospi(x, &w.im, &w.re);
  return w;
}

// Position of element n of a real line in the reordered sequence whose FFT
// gives the DCT-II: even elements first, odd ones reversed at the end.
__device__ __forceinline__ int reorder(int n, int N) { return (n & 1) ? N - 1 - (n >> 1) : (n >> 1); }

// Position in LDS of element e of a complex line of length n: within each
// 16-element row the low bits are XOR-ed with 5 (row mod 4), so that 16
// consecutive lanes meet 16 different banks both on contiguous accesses and
// on the strided writes of the first two radix-4 passes (strides 4 and 16).
// Lines whose length is not a multiple of 16 keep the identity.
__device__ __forceinline__ int swz(int e, int n) { return (n & 15) ? e : e ^ (5 * ((e >> 4) & 3)); }

// Twiddle tables in LDS, filled once per workgroup: W[j] = e^{-2 pi i j/N}
// (the FFT's) and H[k] = e^{-i pi k/(2N)} (the DCT's pre/post factors).
__device__ __forceinline__ void fill_tables(Cx* W, Cx* H, int N) {
  for (int j = threadIdx.x; j < N; j += FDM_NT) {
    W[j] = cispi(-2.0 * (double)j / (double)N);
    H[j] = cispi(-(double)j / (2.0 * N));
  }
}
__device__ __forceinline__ Cx conjc(Cx a) { return {a.re, -a.im}; }

// In-LDS FFTs of `lines` complex lines of length pl.n held in a (line-major);
// b is scratch of the same size.  SIGN -1: forward, +1: inverse (unscaled).
// Returns the buffer holding the result.  Stockham autosort: pass with radix
// r after sub-transforms of length p: butterfly i (k = i mod p) reads
// x[i + q n/r], q < r, multiplies by e^{SIGN 2 pi i q k/(p r)} (entry
// q k n/(p r) of the table W, conjugated for the inverse), takes the length-r
// DFT and writes y[(i - k) r + k + q p].
template <int SIGN>
__device__ Cx* fft_lds(Cx* a, Cx* b, int lines, const FftPlan& pl, const Cx* W, int ls = 0) {
  const int n = pl.n;
  if (ls == 0) ls = n;   // line stride (complex elements)
  int p = 1;
  for (int s = 0; s < pl.nr; ++s) {
    const int r = pl.r[s];
    const int m = n / r;
    const int step = n / (p * r);   // table stride of one unit of k
    for (int t = threadIdx.x; t < lines * m; t += FDM_NT) {
      const int line = t / m, i = t - line * m;
      const int k = i % p;
      const Cx* x = a + line * ls;
      Cx* y = b + line * ls;
      const int j = (i - k) * r + k;
      const int e1 = k * step;
      auto tw = [&](int e) { return SIGN < 0 ? W[e] : conjc(W[e]); };
      if (r == 4) {
        const Cx w1 = tw(e1), w2 = tw(2 * e1), w3 = tw(3 * e1);
        const Cx u0 = x[swz(i, n)], u1 = cmul(x[swz(i + m, n)], w1), u2 = cmul(x[swz(i + 2 * m, n)], w2),
                 u3 = cmul(x[swz(i + 3 * m, n)], w3);
        const Cx s02 = cadd(u0, u2), d02 = csub(u0, u2), s13 = cadd(u1, u3), d13 = cmuli(csub(u1, u3), (double)SIGN);
        y[swz(j, n)] = cadd(s02, s13);
        y[swz(j + p, n)] = cadd(d02, d13);
        y[swz(j + 2 * p, n)] = csub(s02, s13);
        y[swz(j + 3 * p, n)] = csub(d02, d13);
      } else if (r == 2) {
        const Cx u0 = x[swz(i, n)], u1 = cmul(x[swz(i + m, n)], tw(e1));
        y[swz(j, n)] = cadd(u0, u1);
        y[swz(j + p, n)] = csub(u0, u1);
      } else {   // r == 3
        const Cx w1 = tw(e1), w2 = tw(2 * e1);
        const Cx u0 = x[swz(i, n)], u1 = cmul(x[swz(i + m, n)], w1), u2 = cmul(x[swz(i + 2 * m, n)], w2);
        const Cx s12 = cadd(u1, u2);
        // e^{SIGN 2 pi i/3} = -1/2 + SIGN i sqrt(3)/2
        const Cx d12 = cmuli(csub(u1, u2), (double)SIGN * 0.86602540378443864676);
        const Cx c = {u0.re - 0.5 * s12.re, u0.im - 0.5 * s12.im};
        y[swz(j, n)] = cadd(u0, s12);
        y[swz(j + p, n)] = cadd(c, d12);
        y[swz(j + 2 * p, n)] = csub(c, d12);
      }
    }
    __syncthreads();
    Cx* t = a;
    a = b;
    b = t;
    p *= r;
  }
  return a;
}

// DCT-II coefficient k of the real line packed as component `comp` (0: real,
// 1: imaginary) of the complex line whose FFT is Z (length N):
// V = (Z[k] + conj Z[N-k])/2 (comp 0) or (Z[k] - conj Z[N-k])/(2i) (comp 1);
// C[k] = Re(V e^{-i pi k/(2N)}).
__device__ __forceinline__ double dct_coef(const Cx* Z, int k, int N, int comp, const Cx* H) {
  const Cx a = Z[swz(k, N)], b = Z[swz(k == 0 ? 0 : N - k, N)];
  Cx V;
  if (comp == 0) V = {0.5 * (a.re + b.re), 0.5 * (a.im - b.im)};
  else V = {0.5 * (a.im + b.im), -0.5 * (a.re - b.re)};
  const Cx w = H[k];
  return V.re * w.re - V.im * w.im;
}

// Packed inverse spectrum: from the DCT-II coefficients C1, C2 of two real
// lines (R holds them line-major), Z[k] = V1[k] + i V2[k] with
// V[k] = e^{i pi k/(2N)} (C[k] - i C[N-k]), V[0] = C[0].
__device__ __forceinline__ Cx packed_inverse(const double* C1, const double* C2, int k, int N, const Cx* H) {
  Cx V1, V2;
  if (k == 0) {
    V1 = {C1[0], 0.0};
    V2 = {C2[0], 0.0};
  } else {
    const Cx w = conjc(H[k]);
    V1 = {w.re * C1[k] + w.im * C1[N - k], w.im * C1[k] - w.re * C1[N - k]};
    V2 = {w.re * C2[k] + w.im * C2[N - k], w.im * C2[k] - w.re * C2[N - k]};
  }
  return {V1.re - V2.im, V1.im + V2.re};
}

// One-dimensional eigenvalue (unit spacing) of mode k: DST-II basis (both
// faces at phi = 0) or DCT-II basis (both without flux).
__device__ __forceinline__ double lam(int k, int N, int dst) {
  const double s = sinpi((double)(dst ? k + 1 : k) / (2.0 * N));
  return 4.0 * s * s;
}

struct FdmLat {
  int N;            // transform length along the axis
  int dst;          // 1: phi = 0 faces (DST-II), 0: walls (DCT-II)
  long long sline;  // element stride along the axis
  long long so;     // stride of the other lateral index
  int nz;           // z extent (16 consecutive z per workgroup)
  int nzc;          // z chunks
  FftPlan pl;
};

// Forward (INV = false) or inverse transform of every line along one lateral
// axis.  Workgroup: one value of the other lateral index, 16 consecutive z
// (128-byte rows for the loads and stores); 8 complex lines in LDS.
template <bool INV>
__global__ void __launch_bounds__(FDM_NT) k_fdm_lateral(FdmLat A, const double* __restrict__ src,
                                                       double* __restrict__ dst) {
  extern __shared__ Cx lds[];
  const int N = A.N;
  constexpr int L = FDM_LAT_LINES, P = L / 2;
  Cx* bufa = lds;
  Cx* bufb = lds + P * N;
  Cx* W = lds + 2 * P * N;
  Cx* H = W + N;
  fill_tables(W, H, N);
  const int o = blockIdx.x / A.nzc, kc = blockIdx.x - o * A.nzc;
  const int k0 = kc * L;
  const long long base = (long long)o * A.so + k0;
  if (!INV) {
    for (int e = threadIdx.x; e < N * L; e += FDM_NT) {
      const int n = e / L, kk = e - n * L;
      double v = (k0 + kk < A.nz) ? src[base + n * A.sline + kk] : 0.0;
      if (A.dst && (n & 1)) v = -v;
      double* slot = reinterpret_cast<double*>(&bufa[(kk >> 1) * N + swz(reorder(n, N), N)]);
      slot[kk & 1] = v;
    }
    __syncthreads();
    const Cx* Z = fft_lds<-1>(bufa, bufb, P, A.pl, W);
    for (int e = threadIdx.x; e < N * L; e += FDM_NT) {
      const int k = e / L, kk = e - k * L;
      if (k0 + kk >= A.nz) continue;
      const double c = dct_coef(Z + (kk >> 1) * N, k, N, kk & 1, H);
      dst[base + (long long)(A.dst ? N - 1 - k : k) * A.sline + kk] = c;
    }
  } else {
    double* R = reinterpret_cast<double*>(bufb);   // coefficients, line-major (L lines of N)
    for (int e = threadIdx.x; e < N * L; e += FDM_NT) {
      const int n = e / L, kk = e - n * L;
      const double v = (k0 + kk < A.nz) ? src[base + n * A.sline + kk] : 0.0;
      R[kk * N + (A.dst ? N - 1 - n : n)] = v;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < N * P; e += FDM_NT) {
      const int line = e / N, k = e - line * N;
      bufa[line * N + swz(k, N)] = packed_inverse(R + 2 * line * N, R + (2 * line + 1) * N, k, N, H);
    }
    __syncthreads();
    const Cx* z = fft_lds<1>(bufa, bufb, P, A.pl, W);
    const double inv = 1.0 / N;
    for (int e = threadIdx.x; e < N * L; e += FDM_NT) {
      const int n = e / L, kk = e - n * L;
      if (k0 + kk >= A.nz) continue;
      const Cx zv = z[(kk >> 1) * N + swz(reorder(n, N), N)];
      double v = ((kk & 1) ? zv.im : zv.re) * inv;
      if (A.dst && (n & 1)) v = -v;
      dst[base + n * A.sline + kk] = v;
    }
  }
}

// Pipelined form of the lateral pass: persistent workgroups (tables filled
// once) walk the (other index, z chunk) groups with a grid stride; each
// thread holds its FDM_PF elements of the next group in registers, loaded
// while the current group is transformed.  Needs N * 16 <= FDM_PF * FDM_NT.
constexpr int FDM_PF = 24;

template <bool INV>
__global__ void __launch_bounds__(FDM_NT) k_fdm_lateral_pipe(FdmLat A, const double* __restrict__ src,
                                                            double* __restrict__ dst, int ngroups) {
  extern __shared__ Cx lds[];
  const int N = A.N;
  constexpr int L = FDM_LAT_LINES, P = L / 2;
  // lines padded by one element (coefficient rows by one double): lanes that step over lines
  // meet other LDS banks
  const int LS = N + 1, RS = N + 1;
  Cx* bufa = lds;
  Cx* bufb = lds + P * LS;
  Cx* W = lds + 2 * P * LS;
  Cx* H = W + N;
  fill_tables(W, H, N);   // read after the first barrier below
  const int NL = N * L;
  double pf[FDM_PF];
  auto fetch = [&](int grp) {
    const int o = grp / A.nzc, k0 = (grp - o * A.nzc) * L;
    const long long base = (long long)o * A.so + k0;
#pragma unroll
    for (int q = 0; q < FDM_PF; ++q) {
      const int e = threadIdx.x + q * FDM_NT;
      const int n = e / L, kk = e - n * L;
      pf[q] = (e < NL && k0 + kk < A.nz) ? src[base + n * A.sline + kk] : 0.0;
    }
  };
  if ((int)blockIdx.x < ngroups) fetch(blockIdx.x);
  for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const int o = grp / A.nzc, k0 = (grp - o * A.nzc) * L;
    const long long base = (long long)o * A.so + k0;
    double* R = reinterpret_cast<double*>(bufb);   // inverse: coefficients, line-major (L lines of RS)
#pragma unroll
    for (int q = 0; q < FDM_PF; ++q) {
      const int e = threadIdx.x + q * FDM_NT;
      if (e < NL) {
        const int n = e / L, kk = e - n * L;
        if (INV) {
          R[kk * RS + (A.dst ? N - 1 - n : n)] = pf[q];
        } else {
          const double v = (A.dst && (n & 1)) ? -pf[q] : pf[q];
          reinterpret_cast<double*>(&bufa[(kk >> 1) * LS + swz(reorder(n, N), N)])[kk & 1] = v;
        }
      }
    }
    __syncthreads();
    if (grp + (int)gridDim.x < ngroups) fetch(grp + gridDim.x);   // in flight during the transform
    if (!INV) {
      const Cx* Z = fft_lds<-1>(bufa, bufb, P, A.pl, W, LS);
      for (int e = threadIdx.x; e < NL; e += FDM_NT) {
        const int k = e / L, kk = e - k * L;
        if (k0 + kk >= A.nz) continue;
        const double c = dct_coef(Z + (kk >> 1) * LS, k, N, kk & 1, H);
        dst[base + (long long)(A.dst ? N - 1 - k : k) * A.sline + kk] = c;
      }
    } else {
      for (int e = threadIdx.x; e < N * P; e += FDM_NT) {
        const int line = e / N, k = e - line * N;
        bufa[line * LS + swz(k, N)] = packed_inverse(R + 2 * line * RS, R + (2 * line + 1) * RS, k, N, H);
      }
      __syncthreads();
      const Cx* z = fft_lds<1>(bufa, bufb, P, A.pl, W, LS);
      const double inv = 1.0 / N;
      for (int e = threadIdx.x; e < NL; e += FDM_NT) {
        const int n = e / L, kk = e - n * L;
        if (k0 + kk >= A.nz) continue;
        const Cx zv = z[(kk >> 1) * LS + swz(reorder(n, N), N)];
        double v = ((kk & 1) ? zv.im : zv.re) * inv;
        if (A.dst && (n & 1)) v = -v;
        dst[base + n * A.sline + kk] = v;
      }
    }
    __syncthreads();   // this group's LDS reads are done before the next group's writes
  }
}

struct FdmZ {
  int nz;           // cells along z
  int M;            // transform length: nz, or 2 nz for the mirrored line
  int mirror;       // 1: no flux at z- (line mirrored about the z- face)
  int lines;        // real lines per workgroup
  long long nlines; // nx ny
  int ny, nx;
  int dstx, dsty;   // lateral bases
  double scale;     // 1/c_op
  FftPlan pl;
};

// The z part of the solve on contiguous z-lines (lines (i, j) hold the
// lateral mode (i, j) after the lateral forward passes): DST-II of the line
// (or of its mirror image), division of coefficient k by
// c_op (l_x(i) + l_y(j) + l_z(k)), inverse DST-II, in place.
__global__ void __launch_bounds__(FDM_NT) k_fdm_z(FdmZ A, double* __restrict__ x) {
  extern __shared__ Cx lds[];
  const int M = A.M, nz = A.nz, L = A.lines, P = L / 2;
  Cx* bufa = lds;
  Cx* bufb = lds + P * M;
  Cx* W = lds + 2 * P * M;
  Cx* H = W + M;
  fill_tables(W, H, M);
  const long long l0 = (long long)blockIdx.x * L;
  const int nl = (int)(A.nlines - l0 < L ? A.nlines - l0 : L);
  double* line0 = x + l0 * nz;
  // load (contiguous block of nl lines), DST sign and reorder; the mirror puts
  // x[k] at m = nz + k and m = nz - 1 - k
  for (int e = threadIdx.x; e < L * M; e += FDM_NT) {   // zero the lines past the grid
    const int line = e / M;
    if (line >= nl) reinterpret_cast<double*>(&bufa[(line >> 1) * M + (e - line * M)])[line & 1] = 0.0;
  }
  for (int e = threadIdx.x; e < nl * nz; e += FDM_NT) {
    const int line = e / nz, k = e - line * nz;
    const double v = line0[e];
    double* row = reinterpret_cast<double*>(&bufa[(line >> 1) * M]);
    const int c = line & 1;
    if (A.mirror) {
      const int m1 = nz + k, m2 = nz - 1 - k;
      row[2 * swz(reorder(m1, M), M) + c] = (m1 & 1) ? -v : v;
      row[2 * swz(reorder(m2, M), M) + c] = (m2 & 1) ? -v : v;
    } else {
      row[2 * swz(reorder(k, M), M) + c] = (k & 1) ? -v : v;
    }
  }
  __syncthreads();
  const Cx* Z = fft_lds<-1>(bufa, bufb, P, A.pl, W);
  // R = coefficients divided by the eigenvalue sums, in the DCT-II order of the
  // inverse (C'[m] = S[M-1-m] / eigenvalue of DST mode M-1-m)
  double* R = reinterpret_cast<double*>(Z == bufa ? bufb : bufa);
  for (int e = threadIdx.x; e < L * M; e += FDM_NT) {
    const int line = e / M, m = e - line * M;
    double v = 0.0;
    if (line < nl) {
      const long long L_ = l0 + line;
      const int i = (int)(L_ / A.ny), j = (int)(L_ - (long long)i * A.ny);
      const double sig = lam(i, A.nx, A.dstx) + lam(j, A.ny, A.dsty) + lam(M - 1 - m, M, 1);
      v = dct_coef(Z + (line >> 1) * M, m, M, line & 1, H) * A.scale / sig;
    }
    R[line * M + m] = v;
  }
  __syncthreads();
  Cx* Wb = const_cast<Cx*>(Z);
  for (int e = threadIdx.x; e < P * M; e += FDM_NT) {
    const int pr = e / M, k = e - pr * M;
    Wb[pr * M + swz(k, M)] = packed_inverse(R + 2 * pr * M, R + (2 * pr + 1) * M, k, M, H);
  }
  __syncthreads();
  const Cx* z = fft_lds<1>(Wb, reinterpret_cast<Cx*>(R), P, A.pl, W);
  const double inv = 1.0 / M;
  const int off = A.mirror ? nz : 0;
  for (int e = threadIdx.x; e < nl * nz; e += FDM_NT) {
    const int line = e / nz, k = e - line * nz;
    const int m = off + k;
    const Cx zv = z[(line >> 1) * M + swz(reorder(m, M), M)];
    const double v = ((line & 1) ? zv.im : zv.re) * inv;
    line0[e] = (m & 1) ? -v : v;
  }
}

// Pipelined form of the z pass: persistent workgroups walk the blocks of
// `lines` z-lines with a grid stride, each thread holding its FDM_PF
// elements of the next block in registers while the current one is solved.
// Needs lines * nz <= FDM_PF * FDM_NT.
__global__ void __launch_bounds__(FDM_NT) k_fdm_z_pipe(FdmZ A, double* __restrict__ x, int ngroups) {
  extern __shared__ Cx lds[];
  const int M = A.M, nz = A.nz, L = A.lines, P = L / 2;
  Cx* bufa = lds;
  Cx* bufb = lds + P * M;
  Cx* W = lds + 2 * P * M;
  Cx* H = W + M;
  fill_tables(W, H, M);   // read after the first barrier below
  // z eigenvalue of DST mode M-1-m at entry m; the lateral eigenvalue sum of each line of a block
  double* lamz = reinterpret_cast<double*>(H + M);
  double* lxy = lamz + M;
  for (int m = threadIdx.x; m < M; m += FDM_NT) lamz[m] = lam(M - 1 - m, M, 1);
  double pf[FDM_PF];
  auto fetch = [&](int grp) {
    const long long l0 = (long long)grp * L;
    const int nl = (int)(A.nlines - l0 < L ? A.nlines - l0 : L);
    const double* line0 = x + l0 * nz;
#pragma unroll
    for (int q = 0; q < FDM_PF; ++q) {
      const int e = threadIdx.x + q * FDM_NT;
      pf[q] = e < nl * nz ? line0[e] : 0.0;
    }
  };
  if ((int)blockIdx.x < ngroups) fetch(blockIdx.x);
  for (int grp = blockIdx.x; grp < ngroups; grp += gridDim.x) {
    const long long l0 = (long long)grp * L;
    const int nl = (int)(A.nlines - l0 < L ? A.nlines - l0 : L);
    double* line0 = x + l0 * nz;
    if ((int)threadIdx.x < nl) {
      const long long L_ = l0 + threadIdx.x;
      const int i = (int)(L_ / A.ny), j = (int)(L_ - (long long)i * A.ny);
      lxy[threadIdx.x] = lam(i, A.nx, A.dstx) + lam(j, A.ny, A.dsty);
    }
    if (nl < L)
      for (int e = threadIdx.x; e < L * M; e += FDM_NT) {   // zero the lines past the grid
        const int line = e / M;
        if (line >= nl) reinterpret_cast<double*>(&bufa[(line >> 1) * M + (e - line * M)])[line & 1] = 0.0;
      }
#pragma unroll
    for (int q = 0; q < FDM_PF; ++q) {
      const int e = threadIdx.x + q * FDM_NT;
      if (e < nl * nz) {
        const int line = e / nz, k = e - line * nz;
        const double v = pf[q];
        double* row = reinterpret_cast<double*>(&bufa[(line >> 1) * M]);
        const int c = line & 1;
        if (A.mirror) {
          const int m1 = nz + k, m2 = nz - 1 - k;
          row[2 * swz(reorder(m1, M), M) + c] = (m1 & 1) ? -v : v;
          row[2 * swz(reorder(m2, M), M) + c] = (m2 & 1) ? -v : v;
        } else {
          row[2 * swz(reorder(k, M), M) + c] = (k & 1) ? -v : v;
        }
      }
    }
    __syncthreads();
    if (grp + (int)gridDim.x < ngroups) fetch(grp + gridDim.x);   // in flight during the solve
    const Cx* Z = fft_lds<-1>(bufa, bufb, P, A.pl, W);
    double* R = reinterpret_cast<double*>(Z == bufa ? bufb : bufa);
    for (int e = threadIdx.x; e < L * M; e += FDM_NT) {
      const int line = e / M, m = e - line * M;
      double v = 0.0;
      if (line < nl) {
        const double sig = lxy[line] + lamz[m];
        v = dct_coef(Z + (line >> 1) * M, m, M, line & 1, H) * A.scale / sig;
      }
      R[line * M + m] = v;
    }
    __syncthreads();
    Cx* Wb = const_cast<Cx*>(Z);
    for (int e = threadIdx.x; e < P * M; e += FDM_NT) {
      const int pr = e / M, k = e - pr * M;
      Wb[pr * M + swz(k, M)] = packed_inverse(R + 2 * pr * M, R + (2 * pr + 1) * M, k, M, H);
    }
    __syncthreads();
    const Cx* z = fft_lds<1>(Wb, reinterpret_cast<Cx*>(R), P, A.pl, W);
    const double inv = 1.0 / M;
    const int off = A.mirror ? nz : 0;
    for (int e = threadIdx.x; e < nl * nz; e += FDM_NT) {
      const int line = e / nz, k = e - line * nz;
      const int m = off + k;
      const Cx zv = z[(line >> 1) * M + swz(reorder(m, M), M)];
      const double v = ((line & 1) ? zv.im : zv.re) * inv;
      line0[e] = (m & 1) ? -v : v;
    }
    __syncthreads();   // this block's LDS reads are done before the next block's writes
  }
}

struct FdmGeometry {
  bool ok = false;
  FdmLat ax, ay;
  FdmZ az;
  size_t lds_lat_x = 0, lds_lat_y = 0, lds_z = 0;
};

FdmGeometry geometry(const DevParams& P, double c_op) {
  FdmGeometry G;
  // lateral faces in pairs: both walls (DCT) or both at phi = 0 (DST)
  const int kx0 = P.kind[0], kx1 = P.kind[1], ky0 = P.kind[2], ky1 = P.kind[3], kz0 = P.kind[4], kz1 = P.kind[5];
  const bool dx0 = pressure_dirichlet(kx0), dx1 = pressure_dirichlet(kx1);
  const bool dy0 = pressure_dirichlet(ky0), dy1 = pressure_dirichlet(ky1);
  const bool dz0 = pressure_dirichlet(kz0), dz1 = pressure_dirichlet(kz1);
  if (dx0 != dx1 || dy0 != dy1 || !dz1) return G;   // z+ must hold phi = 0
  FdmLat ax, ay;
  ax.N = P.nx;
  ax.dst = dx0;
  ax.sline = (long long)P.ny * P.nz;
  ax.so = P.nz;
  ay.N = P.ny;
  ay.dst = dy0;
  ay.sline = P.nz;
  ay.so = (long long)P.ny * P.nz;
  for (FdmLat* a : {&ax, &ay}) {
    a->nz = P.nz;
    a->nzc = (P.nz + FDM_LAT_LINES - 1) / FDM_LAT_LINES;
    if (!make_plan(a->N, a->pl)) return G;
  }
  FdmZ az;
  az.nz = P.nz;
  az.mirror = dz0 ? 0 : 1;
  az.M = az.mirror ? 2 * P.nz : P.nz;
  if (!make_plan(az.M, az.pl)) return G;
  az.nlines = (long long)P.nx * P.ny;
  az.nx = P.nx;
  az.ny = P.ny;
  az.dstx = ax.dst;
  az.dsty = ay.dst;
  az.scale = 1.0 / c_op;
  // LDS: two complex buffers of the packed lines
  const size_t lmax = 160 * 1024;
  az.lines = 16;
  while (az.lines > 2 && (size_t)(az.lines + 2) * az.M * sizeof(Cx) + (size_t)(az.M + az.lines) * sizeof(double) > lmax)
    az.lines /= 2;
  // two buffers of lines/2 complex lines, two tables; the pipelined z pass also the eigenvalue tables
  G.lds_z = (size_t)(az.lines + 2) * az.M * sizeof(Cx) + (size_t)(az.M + az.lines) * sizeof(double);
  // (the pipelined lateral pass pads each of its 16 half-lines by one element)
  G.lds_lat_x = (size_t)(FDM_LAT_LINES + 2) * ax.N * sizeof(Cx) + FDM_LAT_LINES * sizeof(Cx);
  G.lds_lat_y = (size_t)(FDM_LAT_LINES + 2) * ay.N * sizeof(Cx) + FDM_LAT_LINES * sizeof(Cx);
  if (G.lds_z > lmax || G.lds_lat_x > lmax || G.lds_lat_y > lmax) return G;
  G.ax = ax;
  G.ay = ay;
  G.az = az;
  G.ok = true;
  return G;
}

}  // namespace

bool fdm_supported(const DevParams& P) { return geometry(P, 1.0).ok; }

int launch_fdm_solve(const DevParams& P, double c_op, const double* b, double* x, double* t, hipStream_t s) {
  const FdmGeometry G = geometry(P, c_op);
  if (!G.ok) return -1;
  static bool attr = false;
  if (!attr) {
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_fdm_lateral<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_fdm_lateral<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_fdm_z), hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_fdm_z_pipe), hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_fdm_lateral_pipe<false>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    (void)hipFuncSetAttribute(reinterpret_cast<const void*>(k_fdm_lateral_pipe<true>),
                              hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    attr = true;
  }
  const int gx = P.ny * G.ax.nzc, gy = P.nx * G.ay.nzc;
  const int gz = (int)((G.az.nlines + G.az.lines - 1) / G.az.lines);
  // persistent grid of the pipelined lateral passes: as many workgroups as
  // the compute units hold at once
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                              hipSuccess)
    return -1;
  auto lateral = [&](bool inv, const FdmLat& a, size_t lds, int groups, const double* in, double* out) {
    if (a.N * FDM_LAT_LINES <= FDM_PF * FDM_NT) {
      const int per_cu = (int)std::max<size_t>(1, (160 * 1024) / lds);
      const int nb = std::min(groups, per_cu * ncu);
      if (inv) k_fdm_lateral_pipe<true><<<nb, FDM_NT, lds, s>>>(a, in, out, groups);
      else k_fdm_lateral_pipe<false><<<nb, FDM_NT, lds, s>>>(a, in, out, groups);
    } else if (inv) {
      k_fdm_lateral<true><<<groups, FDM_NT, lds, s>>>(a, in, out);
    } else {
      k_fdm_lateral<false><<<groups, FDM_NT, lds, s>>>(a, in, out);
    }
  };
  // b -> t (x), t -> x (y), z solve in x, x -> t (y), t -> x (x)
  lateral(false, G.ax, G.lds_lat_x, gx, b, t);
  lateral(false, G.ay, G.lds_lat_y, gy, t, x);
  if (G.az.lines * G.az.nz <= FDM_PF * FDM_NT) {
    const int per_cu = (int)std::max<size_t>(1, (160 * 1024) / G.lds_z);
    k_fdm_z_pipe<<<std::min(gz, per_cu * ncu), FDM_NT, G.lds_z, s>>>(G.az, x, gz);
  } else {
    k_fdm_z<<<gz, FDM_NT, G.lds_z, s>>>(G.az, x);
  }
  lateral(true, G.ay, G.lds_lat_y, gy, x, t);
  lateral(true, G.ax, G.lds_lat_x, gx, t, x);
  return 0;
}

}  // namespace dsv
