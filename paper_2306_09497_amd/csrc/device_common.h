// Device-side constants and helpers shared by the kernels: tile shapes,
// index maps, complex arithmetic, the recurrence coefficients of the
// normalised Legendre functions and the per-m coefficients of the linear
// operator.  Kept apart from the host-side declarations so that what the
// kernels compile against is one file.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace pint {

constexpr int kSynFields = 6;
constexpr int kAnaFields = 4;
constexpr int kMaxNlon = 1024;
constexpr int kGemmTR = 64;      // Legendre GEMM tile rows (synthesis)
constexpr int kGemmTRAnal = 32;  // Legendre GEMM tile rows per parity (analysis)
constexpr int kGemmTC = 64;      // Legendre GEMM tile columns
constexpr int kGemmTK = 16;      // Legendre GEMM k-slab staged in LDS
constexpr int kRingThreads = 512;

inline __host__ __device__ int coef_idx(int M, int m, int n) {
  return m * (2 * M + 3 - m) / 2 + (n - m);
}

// Pitch, in elements of type E, between the rows of wavenumbers m and m + 1
// of the Fourier arrays F[m][latitude][column] and G (ncol columns per
// latitude).  nlat * ncol alone is a multiple of 256 KiB at batched sizes
// (T255, 64 states: 9 x 256 KiB), which puts every wavenumber row that one
// ring reads at the same L2 set and channel; 256 bytes of padding spread
// them over the channels.
constexpr int kFourierPadBytes = 256;
template <typename E>
__host__ __device__ inline size_t fourier_pitch(int nlat, int ncol) {
  return (size_t)nlat * ncol + kFourierPadBytes / sizeof(E);
}

// ---- small device helpers shared by the kernels ----
// Workgroups are dispatched round-robin over the 8 XCDs (block L on XCD L mod
// 8), each with its own L2.  Remap the hardware block index so that every XCD
// works through one contiguous range of logical blocks: logically adjacent
// blocks (which share operand rows) then share an L2.
constexpr int kNumXcd = 8;
__device__ inline int xcd_remap(int L, int T) {
  const int q = T / kNumXcd, r = T % kNumXcd;
  const int x = L % kNumXcd, i = L / kNumXcd;
  return x * q + (x < r ? x : r) + i;
}

__device__ inline double2 cmul(double2 x, double2 y) {
  return make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}
__device__ inline float2 cmul(float2 x, float2 y) {
  return make_float2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}
__device__ inline double2 cinv(double2 x) {
  const double d = x.x * x.x + x.y * x.y;
  return make_double2(x.x / d, -x.y / d);
}

// eps_n^m = sqrt((n^2 - m^2) / (4 n^2 - 1)), zero for n <= m
__device__ inline double eps_nm(int n, int m) {
  if (n <= m) return 0.0;
  return sqrt(((double)n * n - (double)m * m) / (4.0 * n * n - 1.0));
}

// inverse-Laplacian factor: psi_k = s_k xi_k, s_k = -a^2/(k(k+1)), s_0 = 0
__device__ inline double s_of(int k, double a) {
  return k > 0 ? -a * a / ((double)k * (k + 1)) : 0.0;
}


// Coefficients of the linear operator in the per-m chain form (see cn_factors).
struct CnCoef {
  double A, B, C, lap;
};

__device__ inline CnCoef cn_coef(int m, int n, int M, double a, double W, bool lg) {
  CnCoef c;
  const double Wa = W / (a * a);
  const double en = eps_nm(n, m);
  c.A = -W * en + Wa * (n - 1) * en * s_of(n - 1, a);
  c.B = -Wa * m * s_of(n, a);
  if (n < M) {
    const double e1 = eps_nm(n + 1, m);
    c.C = -W * e1 - Wa * (n + 2) * e1 * s_of(n + 1, a);
  } else {
    c.C = 0.0;
  }
  c.lap = lg ? (double)n * (n + 1) / (a * a) : 0.0;
  return c;
}

}  // namespace pint
