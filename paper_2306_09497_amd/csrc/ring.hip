// Latitude-ring kernels: the FFT half of the spectral transform (Sec. 2.2)
// fused with the pointwise nonlinear terms (Sec. 2.1, A-grid pseudospectral
// evaluation).  One workgroup per (latitude j, state b); the ring lives in LDS.
//
// Real signals are transformed in pairs through one complex FFT (x + i y).
// The FFT is a mixed-radix (4, 2, 3, 5) Stockham transform in a single LDS
// buffer per signal: each pass loads its butterflies' operands into
// registers, synchronises, then writes the butterfly outputs.
#include "pint_internal.h"

namespace pint {

__device__ inline double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 c_sub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 c_scl(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// multiply by sign * i
__device__ inline double2 c_si(double2 a, double sign) { return make_double2(-sign * a.y, sign * a.x); }

// In-register DFT of size R: y_k = sum_r v_r exp(sign 2 pi i r k / R).
template <int R>
__device__ inline void dft(double2* v, double sign);

template <>
__device__ inline void dft<2>(double2* v, double) {
  const double2 a = v[0], b = v[1];
  v[0] = c_add(a, b);
  v[1] = c_sub(a, b);
}

template <>
__device__ inline void dft<3>(double2* v, double sign) {
  const double h = 0.86602540378443864676;   // sin(2 pi / 3)
  const double2 t = c_add(v[1], v[2]);
  const double2 d = c_sub(v[1], v[2]);
  const double2 base = c_sub(v[0], c_scl(t, 0.5));
  const double2 rot = c_si(c_scl(d, h), sign);
  v[0] = c_add(v[0], t);
  v[1] = c_add(base, rot);
  v[2] = c_sub(base, rot);
}

template <>
__device__ inline void dft<4>(double2* v, double sign) {
  const double2 s02 = c_add(v[0], v[2]), d02 = c_sub(v[0], v[2]);
  const double2 s13 = c_add(v[1], v[3]), d13 = c_si(c_sub(v[1], v[3]), sign);
  v[0] = c_add(s02, s13);
  v[2] = c_sub(s02, s13);
  v[1] = c_add(d02, d13);
  v[3] = c_sub(d02, d13);
}

template <>
__device__ inline void dft<5>(double2* v, double sign) {
  const double c1 = 0.30901699437494742410, c2 = -0.80901699437494742410;   // cos(2pi/5), cos(4pi/5)
  const double s1 = 0.95105651629515357212, s2 = 0.58778525229247312917;    // sin(2pi/5), sin(4pi/5)
  const double2 a1 = c_add(v[1], v[4]), a2 = c_add(v[2], v[3]);
  const double2 b1 = c_sub(v[1], v[4]), b2 = c_sub(v[2], v[3]);
  const double2 y0 = c_add(v[0], c_add(a1, a2));
  const double2 r1 = c_add(v[0], c_add(c_scl(a1, c1), c_scl(a2, c2)));
  const double2 r2 = c_add(v[0], c_add(c_scl(a1, c2), c_scl(a2, c1)));
  const double2 i1 = c_si(c_add(c_scl(b1, s1), c_scl(b2, s2)), sign);
  const double2 i2 = c_si(c_sub(c_scl(b1, s2), c_scl(b2, s1)), sign);
  v[0] = y0;
  v[1] = c_add(r1, i1);
  v[4] = c_sub(r1, i1);
  v[2] = c_add(r2, i2);
  v[3] = c_sub(r2, i2);
}

// exp(i 2 pi t / 16) from cos(pi/8), sin(pi/8) and sqrt(1/2) by octant
// symmetry (t taken mod 16).
struct C2 {
  double c, s;
};
constexpr C2 w16(int t) {
  const double a = 0.92387953251128675613, b = 0.38268343236508977173,
               h = 0.70710678118654752440;
  const C2 q0[4] = {{1.0, 0.0}, {a, b}, {h, h}, {b, a}};   // first quadrant, t = 0..3
  t = ((t % 16) + 16) % 16;
  const C2 v = q0[t % 4];
  switch (t / 4) {        // rotate by i^(t/4)
    case 0: return v;
    case 1: return {-v.s, v.c};
    case 2: return {-v.c, -v.s};
    default: return {v.s, -v.c};
  }
}

// v * exp(sign 2 pi i T / R) for a compile-time T, R in {2, 4, 8, 16}; the
// multiples of pi/2 cost no multiplication.
template <int R, int T>
__device__ inline double2 mul_w(double2 v, double sign) {
  constexpr int t = (T * (16 / R)) % 16;
  if constexpr (t == 0) {
    return v;
  } else if constexpr (t == 4) {
    return c_si(v, sign);
  } else if constexpr (t == 8) {
    return make_double2(-v.x, -v.y);
  } else if constexpr (t == 12) {
    return c_si(v, -sign);
  } else {
    constexpr C2 w = w16(t);
    const double ws = sign * w.s;
    return make_double2(v.x * w.c - v.y * ws, v.x * ws + v.y * w.c);
  }
}

// In-register DFT of size R1 * R2 by one Cooley-Tukey split: inner DFTs of
// size R2 over v[n1 + R1 n2], twiddles exp(sign 2 pi i n1 k2 / R), outer DFTs
// of size R1; output index k2 + R2 k1.
template <int R1, int R2, int N1 = 0>
__device__ inline void split_inner(double2 (&u)[R1][R2], const double2* v, double sign) {
  if constexpr (N1 < R1) {
    double2 t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = v[N1 + R1 * n2];
    dft<R2>(t, sign);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) u[N1][k2] = t[k2];
    split_inner<R1, R2, N1 + 1>(u, v, sign);
  }
}

template <int R1, int R2, int N1 = 1, int K2 = 1>
__device__ inline void split_twiddle(double2 (&u)[R1][R2], double sign) {
  if constexpr (N1 < R1) {
    if constexpr (K2 < R2) {
      u[N1][K2] = mul_w<R1 * R2, N1 * K2>(u[N1][K2], sign);
      split_twiddle<R1, R2, N1, K2 + 1>(u, sign);
    } else {
      split_twiddle<R1, R2, N1 + 1, 1>(u, sign);
    }
  }
}

template <int R1, int R2>
__device__ inline void dft_split(double2* v, double sign) {
  double2 u[R1][R2];
  split_inner<R1, R2>(u, v, sign);
  split_twiddle<R1, R2>(u, sign);
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    double2 t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = u[n1][k2];
    dft<R1>(t, sign);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) v[k2 + R2 * k1] = t[k1];
  }
}

template <>
__device__ inline void dft<8>(double2* v, double sign) { dft_split<2, 4>(v, sign); }

template <>
__device__ inline void dft<16>(double2* v, double sign) { dft_split<4, 4>(v, sign); }

// ---- compile-time FFT plan for a ring of N points: radix-16 passes first,
// then 8, 4, 2, then radix-3 and radix-5 passes ----
constexpr int fft_npass(int N) {
  int c = 0;
  while (N % 16 == 0) { N /= 16; ++c; }
  while (N % 8 == 0) { N /= 8; ++c; }
  while (N % 4 == 0) { N /= 4; ++c; }
  while (N % 2 == 0) { N /= 2; ++c; }
  while (N % 3 == 0) { N /= 3; ++c; }
  while (N % 5 == 0) { N /= 5; ++c; }
  return c;
}
constexpr int fft_radix(int N, int i) {
  int c = 0;
  while (N % 16 == 0) { if (c++ == i) return 16; N /= 16; }
  while (N % 8 == 0) { if (c++ == i) return 8; N /= 8; }
  while (N % 4 == 0) { if (c++ == i) return 4; N /= 4; }
  while (N % 2 == 0) { if (c++ == i) return 2; N /= 2; }
  while (N % 3 == 0) { if (c++ == i) return 3; N /= 3; }
  while (N % 5 == 0) { if (c++ == i) return 5; N /= 5; }
  return 1;
}
constexpr int fft_ns(int N, int i) {       // product of the radices before pass i
  int p = 1;
  for (int k = 0; k < i; ++k) p *= fft_radix(N, k);
  return p;
}

// LDS layout of a ring buffer: signal s, point i at s * SP + i + i/16 (one
// pad slot per 16 points breaks the power-of-two strides of the early
// Stockham passes across the LDS banks).
template <int N>
struct RingLds {
  static constexpr int SP = N + N / 16;
  __device__ static inline int at(int s, int i) { return s * SP + i + (i >> 4); }
};

// One Stockham pass of radix R over NSIG signals: every thread loads the
// operands of its butterflies into registers, the workgroup synchronises,
// then each thread twiddles, transforms and stores its butterflies.
template <int N, int NSIG, int R, int NS>
__device__ inline void fft_pass(double2* buf, double sign, const double2* __restrict__ tw,
                                int tid) {
  constexpr int NB = N / R;
  constexpr int TOTAL = NSIG * NB;
  constexpr int NBF = (TOTAL + kRingThreads - 1) / kRingThreads;
  constexpr int TSTEP = N / (NS * R);
  using L = RingLds<N>;
  double2 v[NBF][R];
#pragma unroll
  for (int t = 0; t < NBF; ++t) {
    const int id = tid + t * kRingThreads;
    if (id < TOTAL) {
      const int sig = id / NB, j = id - sig * NB;
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = buf[L::at(sig, j + r * NB)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < NBF; ++t) {
    const int id = tid + t * kRingThreads;
    if (id < TOTAL) {
      const int sig = id / NB, j = id - sig * NB;
      const int k = j % NS;
      if constexpr (NS > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) {
          double2 w = tw[r * k * TSTEP];        // exp(-2 pi i r k / (NS R))
          if (sign > 0.0) w.y = -w.y;
          v[t][r] = cmul(v[t][r], w);
        }
      }
      dft<R>(v[t], sign);
      const int o = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[L::at(sig, o + r * NS)] = v[t][r];
    }
  }
  __syncthreads();
}

template <int N, int NSIG, int I>
__device__ inline void fft_passes(double2* buf, double sign, const double2* __restrict__ tw,
                                  int tid) {
  if constexpr (I < fft_npass(N)) {
    fft_pass<N, NSIG, fft_radix(N, I), fft_ns(N, I)>(buf, sign, tw, tid);
    fft_passes<N, NSIG, I + 1>(buf, sign, tw, tid);
  }
}

// Complex FFT of NSIG signals in LDS: sign -1 forward, +1 inverse (unnormalised).
// tid: the thread's index among the kRingThreads threads sharing buf.
template <int N, int NSIG>
__device__ inline void fft_lds(double2* buf, double sign, const double2* __restrict__ tw,
                               int tid) {
  static_assert(fft_ns(N, fft_npass(N)) == N, "ring length must be 2^a 3^b 5^c");
  fft_passes<N, NSIG, 0>(buf, sign, tw, tid);
}

// Sum NV per-thread values over the workgroup (fixed order: wave shuffles,
// then the wave partials in LDS).  red must hold kRingWaves * NV doubles.
constexpr int kRingWaves = kRingThreads / 64;
// Waves that hold no data (wave_active == false, uniform per wave) skip the
// cross-lane shuffles.
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* red, int tid, bool wave_active = true) {
  const int lane = tid & 63, wave = tid >> 6;
  if (wave_active) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) red[wave * NV + i] = v[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kRingWaves; ++w) t += red[w * NV + i];
    v[i] = t;
  }
  __syncthreads();
}

// Two real signals share one complex FFT as x + i s y.  FFT rounding is
// relative to the norm of the whole complex signal, so the power of two s
// (exact to apply and to remove) brings y to the magnitude of x; otherwise
// the smaller signal would inherit the rounding of the larger one.
__device__ inline double pair_scale(double nx2, double ny2) {
  if (!(nx2 > 0.0) || !(ny2 > 0.0)) return 1.0;
  int e = (int)lrint(0.5 * log2(nx2 / ny2));
  e = e < -600 ? -600 : (e > 600 ? 600 : e);
  return ldexp(1.0, e);
}

// Place the spectrum of the real pair (X, Y) (m = 0..M) into z = x + i y:
// Z[m] = X_m + i Y_m, Z[-m] = conj(X_m) + i conj(Y_m); at m = 0 only the
// real parts count (a real field's mean).
template <int N>
__device__ inline void put_pair(double2* z, int sig, int m, double2 X, double2 Y) {
  using L = RingLds<N>;
  if (m == 0) {
    z[L::at(sig, 0)] = make_double2(X.x, Y.x);
  } else {
    z[L::at(sig, m)] = make_double2(X.x - Y.y, X.y + Y.x);
    z[L::at(sig, N - m)] = make_double2(X.x + Y.y, Y.x - X.y);
  }
}

// Split Z = FFT(x + i y) of two real signals: X_m = (Z_m + conj Z_{-m}) / 2,
// Y_m = (Z_m - conj Z_{-m}) / (2i).
template <int N>
__device__ inline void get_pair(const double2* z, int sig, int m, double2* X, double2* Y) {
  using L = RingLds<N>;
  const double2 zp = z[L::at(sig, m)];
  const double2 zm = z[L::at(sig, m == 0 ? 0 : N - m)];
  *X = make_double2(0.5 * (zp.x + zm.x), 0.5 * (zp.y - zm.y));
  *Y = make_double2(0.5 * (zp.y + zm.y), -0.5 * (zp.x - zm.x));
}

// ---------------------------------------------------------------------------
// Tendency ring kernel.  In: synthesis E/O rows (6 fields: xi, delta, Phi', G,
// U, V).  Grid values: xi, delta, Phi', dPhi'/dlambda (= i m Phi'), G, U, V,
// transformed as the pairs (U, V), (G, dPhi'/dlambda), (xi, delta), (Phi', 0)
// (fields of like magnitude share an FFT).  Pointwise (c^2 = 1 - mu_j^2):
//   N_Phi = -(U dPhi'/dlambda + V G) / (a c^2) - Phi' delta
//   A = xi U / c^2,  B = xi V / c^2,  K = (U^2 + V^2) / (2 c^2)
// each scaled by w_j / nlon, then forward FFT of (N_Phi, K), (A, B), m = 0..M,
// to G[m][j][(b*4+f)*2].
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kRingThreads) __attribute__((amdgpu_waves_per_eu(4))) void k_ring_tendency(
    const double* __restrict__ F, double* __restrict__ Gout, const double* __restrict__ c2,
    const double* __restrict__ w, const double2* __restrict__ tw, int M, int nlat, int nlat2,
    int B, double a) {
  constexpr int nlon = N;
  using L = RingLds<N>;
  extern __shared__ double2 zb[];
  __shared__ double red[kRingWaves * 8];
  // logical block = j * B + b (states of one latitude adjacent: their
  // Fourier rows are contiguous), XCD-remapped
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int j = lb / B, b = lb - j * B;
  const int jn = j < nlat2 ? j : nlat - 1 - j;
  const double sg = j < nlat2 ? 1.0 : -1.0;
  const int ncs = 12 * B;
  const int tid = threadIdx.x;
  auto fourier = [&](int m, double2* v) {
    const double2* e = reinterpret_cast<const double2*>(F + ((size_t)(2 * m) * nlat2 + jn) * ncs + b * 12);
    const double2* o = reinterpret_cast<const double2*>(F + ((size_t)(2 * m + 1) * nlat2 + jn) * ncs + b * 12);
#pragma unroll
    for (int f = 0; f < 6; ++f) v[f] = c_add(e[f], c_scl(o[f], sg));
    v[6] = make_double2(-m * v[2].y, m * v[2].x);     // dPhi'/dlambda = i m Phi'
  };
  // field norms over the ring (Parseval, up to a common factor)
  double nrm[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int m = tid; m <= M; m += kRingThreads) {
    double2 v[7];
    fourier(m, v);
#pragma unroll
    for (int f = 0; f < 7; ++f) nrm[f] += v[f].x * v[f].x + v[f].y * v[f].y;
  }
  block_sum<7>(nrm, red, tid, (tid & ~63) <= M);
  // fields: 0 xi, 1 delta, 2 Phi', 3 G, 4 U, 5 V, 6 dPhi'/dlambda
  const double sUV = pair_scale(nrm[4], nrm[5]);
  const double sGL = pair_scale(nrm[3], nrm[6]);
  const double sXD = pair_scale(nrm[0], nrm[1]);
  for (int i = tid; i < 4 * L::SP; i += kRingThreads) zb[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int m = tid; m <= M; m += kRingThreads) {
    double2 v[7];
    fourier(m, v);                                             // L2 hits
    put_pair<N>(zb, 0, m, v[4], c_scl(v[5], sUV));              // U + i s V
    put_pair<N>(zb, 1, m, v[3], c_scl(v[6], sGL));              // G + i s dPhi'/dlambda
    put_pair<N>(zb, 2, m, v[0], c_scl(v[1], sXD));              // xi + i s delta
    put_pair<N>(zb, 3, m, v[2], make_double2(0.0, 0.0));        // Phi'
  }
  __syncthreads();
  fft_lds<N, 4>(zb, 1.0, tw, tid);
  const double ic2 = 1.0 / c2[j];
  const double sc = w[j] / nlon;
  const double ia = 1.0 / a;
  // the pair scales are exact powers of two: their inverses by exponent flip
  const double iUV = ldexp(1.0, -ilogb(sUV)), iGL = ldexp(1.0, -ilogb(sGL)),
               iXD = ldexp(1.0, -ilogb(sXD));
  constexpr int NPT = (N + kRingThreads - 1) / kRingThreads;   // grid points per thread
  double pv[NPT][4];
  double fn[4] = {0, 0, 0, 0};
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int k = tid + t * kRingThreads;
    if (k < nlon) {
      const double2 z1 = zb[L::at(0, k)], z2 = zb[L::at(1, k)], z3 = zb[L::at(2, k)],
                    z4 = zb[L::at(3, k)];
      const double U = z1.x, V = z1.y * iUV, G = z2.x, phl = z2.y * iGL;
      const double xi = z3.x, de = z3.y * iXD, ph = z4.x;
      const double nphi = (-(U * phl + V * G) * ic2 * ia - ph * de) * sc;
      const double A = xi * U * ic2 * sc, Bv = xi * V * ic2 * sc;
      const double K = 0.5 * (U * U + V * V) * ic2 * sc;
      pv[t][0] = nphi;
      pv[t][1] = K;
      pv[t][2] = A;
      pv[t][3] = Bv;
      fn[0] += nphi * nphi;
      fn[1] += K * K;
      fn[2] += A * A;
      fn[3] += Bv * Bv;
    }
  }
  block_sum<4>(fn, red, tid);      // also orders the reads above before the writes below
  const double sNK = pair_scale(fn[0], fn[1]);
  const double sAB = pair_scale(fn[2], fn[3]);
#pragma unroll
  for (int t = 0; t < NPT; ++t) {
    const int k = tid + t * kRingThreads;
    if (k < nlon) {
      zb[L::at(0, k)] = make_double2(pv[t][0], pv[t][1] * sNK);
      zb[L::at(1, k)] = make_double2(pv[t][2], pv[t][3] * sAB);
    }
  }
  __syncthreads();
  fft_lds<N, 2>(zb, -1.0, tw, tid);
  const int ncg = 8 * B;
  const double iNK = ldexp(1.0, -ilogb(sNK)), iAB = ldexp(1.0, -ilogb(sAB));
  for (int m = tid; m <= M; m += kRingThreads) {
    double2 X0, Y0, X1, Y1;
    get_pair<N>(zb, 0, m, &X0, &Y0);
    get_pair<N>(zb, 1, m, &X1, &Y1);
    double2* g = reinterpret_cast<double2*>(Gout + ((size_t)m * nlat + j) * ncg + b * 8);
    g[0] = X0;
    g[1] = c_scl(Y0, iNK);
    g[2] = X1;
    g[3] = c_scl(Y1, iAB);
  }
}

// ---------------------------------------------------------------------------
// Scalar rings for the public transforms (two states per workgroup).
// synthesis: E/O rows (nf = 1) -> grid[b][j][k]
// analysis:  grid[b][j][k] -> G[m][j][b*2] scaled by w_j / nlon
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kRingThreads) void k_ring_synth(const double* __restrict__ F,
                                                             double* __restrict__ grid,
                                                             const double2* __restrict__ tw,
                                                             int M, int nlat, int nlat2, int B) {
  constexpr int nlon = N;
  using L = RingLds<N>;
  extern __shared__ double2 zb[];
  __shared__ double red[kRingWaves * 2];
  const int j = blockIdx.x, b0 = 2 * blockIdx.y;
  const bool two = b0 + 1 < B;
  const int jn = j < nlat2 ? j : nlat - 1 - j;
  const double sg = j < nlat2 ? 1.0 : -1.0;
  const int ncs = 2 * B;
  auto fourier = [&](int m, double2* x, double2* y) {
    const double2* e = reinterpret_cast<const double2*>(F + ((size_t)(2 * m) * nlat2 + jn) * ncs);
    const double2* o = reinterpret_cast<const double2*>(F + ((size_t)(2 * m + 1) * nlat2 + jn) * ncs);
    *x = c_add(e[b0], c_scl(o[b0], sg));
    *y = two ? c_add(e[b0 + 1], c_scl(o[b0 + 1], sg)) : make_double2(0.0, 0.0);
  };
  double nrm[2] = {0, 0};
  for (int m = threadIdx.x; m <= M; m += kRingThreads) {
    double2 x, y;
    fourier(m, &x, &y);
    nrm[0] += x.x * x.x + x.y * x.y;
    nrm[1] += y.x * y.x + y.y * y.y;
  }
  block_sum<2>(nrm, red, threadIdx.x);
  const double sc = pair_scale(nrm[0], nrm[1]);
  for (int i = threadIdx.x; i < L::SP; i += kRingThreads) zb[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int m = threadIdx.x; m <= M; m += kRingThreads) {
    double2 x, y;
    fourier(m, &x, &y);
    put_pair<N>(zb, 0, m, x, c_scl(y, sc));
  }
  __syncthreads();
  fft_lds<N, 1>(zb, 1.0, tw, threadIdx.x);
  const double isc = 1.0 / sc;
  for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
    const double2 z = zb[L::at(0, k)];
    grid[((size_t)b0 * nlat + j) * nlon + k] = z.x;
    if (two) grid[((size_t)(b0 + 1) * nlat + j) * nlon + k] = z.y * isc;
  }
}

template <int N>
__global__ __launch_bounds__(kRingThreads) void k_ring_anal(const double* __restrict__ grid,
                                                            double* __restrict__ Gout,
                                                            const double* __restrict__ w,
                                                            const double2* __restrict__ tw,
                                                            int M, int nlat, int B) {
  constexpr int nlon = N;
  using L = RingLds<N>;
  extern __shared__ double2 zb[];
  __shared__ double red[kRingWaves * 2];
  const int j = blockIdx.x, b0 = 2 * blockIdx.y;
  const bool two = b0 + 1 < B;
  const double sc = w[j] / nlon;
  double nrm[2] = {0, 0};
  for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
    const double x = grid[((size_t)b0 * nlat + j) * nlon + k];
    const double y = two ? grid[((size_t)(b0 + 1) * nlat + j) * nlon + k] : 0.0;
    nrm[0] += x * x;
    nrm[1] += y * y;
  }
  block_sum<2>(nrm, red, threadIdx.x);
  const double s = pair_scale(nrm[0], nrm[1]);
  for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
    const double x = grid[((size_t)b0 * nlat + j) * nlon + k];
    const double y = two ? grid[((size_t)(b0 + 1) * nlat + j) * nlon + k] : 0.0;
    zb[L::at(0, k)] = make_double2(x * sc, y * s * sc);
  }
  __syncthreads();
  fft_lds<N, 1>(zb, -1.0, tw, threadIdx.x);
  const int ncg = 2 * B;
  const double is = 1.0 / s;
  for (int m = threadIdx.x; m <= M; m += kRingThreads) {
    double2 X, Y;
    get_pair<N>(zb, 0, m, &X, &Y);
    double2* g = reinterpret_cast<double2*>(Gout + ((size_t)m * nlat + j) * ncg);
    g[b0] = X;
    if (two) g[b0 + 1] = c_scl(Y, is);
  }
}

// Ring lengths with a compiled FFT plan.
#define PINT_FOR_EACH_NLON(X) \
  X(64) X(96) X(128) X(192) X(256) X(384) X(512) X(640) X(768) X(1024)

bool ring_supported(int nlon) {
#define PINT_CASE(n) if (nlon == n) return true;
  PINT_FOR_EACH_NLON(PINT_CASE)
#undef PINT_CASE
  return false;
}

// Dynamic LDS of the tendency ring kernel: 4 signals.
size_t ring_lds_bytes(int nlon) {
  switch (nlon) {
#define PINT_CASE(n) \
  case n:            \
    return (size_t)4 * RingLds<n>::SP * sizeof(double2);
    PINT_FOR_EACH_NLON(PINT_CASE)
#undef PINT_CASE
    default:
      return 0;
  }
}

// Allow the tendency ring kernel its dynamic LDS.
pint_status ring_prepare(int nlon) {
  switch (nlon) {
#define PINT_CASE(n)                                                                          \
  case n:                                                                                     \
    PINT_HIP(hipFuncSetAttribute((const void*)k_ring_tendency<n>,                             \
                                 hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                                 (int)ring_lds_bytes(n)));                                    \
    return PINT_OK;
    PINT_FOR_EACH_NLON(PINT_CASE)
#undef PINT_CASE
    default:
      set_error("no ring FFT for nlon=%d", nlon);
      return PINT_E_INVAL;
  }
}

pint_status ring_tendency(Plan& p, int B, hipStream_t s) {
  ProfScope ps(p, PK_RING, B, s);
  switch (p.nlon) {
#define PINT_CASE(n)                                                                         \
  case n:                                                                                    \
    hipLaunchKernelGGL(k_ring_tendency<n>, dim3(p.nlat * B), dim3(kRingThreads),             \
                       ring_lds_bytes(n), s, p.F, p.G, p.c2, p.w, p.twid, p.M, p.nlat,       \
                       p.nlat2, B, p.a);                                                     \
    break;
    PINT_FOR_EACH_NLON(PINT_CASE)
#undef PINT_CASE
    default:
      set_error("no ring FFT for nlon=%d", p.nlon);
      return PINT_E_INVAL;
  }
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status scalar_prep(Plan& p, const double* spec, int B, hipStream_t s);
pint_status scalar_post(Plan& p, double* spec, int B, hipStream_t s);

pint_status scalar_synthesis(Plan& p, const double* spec, double* grid, int B, hipStream_t s) {
  for (int b0 = 0; b0 < B; b0 += p.max_batch) {
    const int nb = (B - b0) < p.max_batch ? (B - b0) : p.max_batch;
    pint_status st = scalar_prep(p, spec + (size_t)b0 * p.ncoef * 2, nb, s);
    if (st != PINT_OK) return st;
    st = legendre_synth(p, nb, 1, s);
    if (st != PINT_OK) return st;
    {
      ProfScope ps(p, PK_SRING, nb, s);
      double* gout = grid + (size_t)b0 * p.nlat * p.nlon;
      switch (p.nlon) {
#define PINT_CASE(n)                                                                             \
  case n:                                                                                        \
    hipLaunchKernelGGL(k_ring_synth<n>, dim3(p.nlat, (nb + 1) / 2), dim3(kRingThreads),          \
                       (size_t)RingLds<n>::SP * sizeof(double2), s, p.F, gout, p.twid, p.M,      \
                       p.nlat, p.nlat2, nb);                                                     \
    break;
        PINT_FOR_EACH_NLON(PINT_CASE)
#undef PINT_CASE
        default:
          set_error("no ring FFT for nlon=%d", p.nlon);
          return PINT_E_INVAL;
      }
      PINT_HIP(hipGetLastError());
    }
  }
  return PINT_OK;
}

pint_status scalar_analysis(Plan& p, const double* grid, double* spec, int B, hipStream_t s) {
  for (int b0 = 0; b0 < B; b0 += p.max_batch) {
    const int nb = (B - b0) < p.max_batch ? (B - b0) : p.max_batch;
    {
      ProfScope ps(p, PK_SRING, nb, s);
      const double* gin = grid + (size_t)b0 * p.nlat * p.nlon;
      switch (p.nlon) {
#define PINT_CASE(n)                                                                            \
  case n:                                                                                       \
    hipLaunchKernelGGL(k_ring_anal<n>, dim3(p.nlat, (nb + 1) / 2), dim3(kRingThreads),          \
                       (size_t)RingLds<n>::SP * sizeof(double2), s, gin, p.G, p.w, p.twid, p.M, \
                       p.nlat, nb);                                                             \
    break;
        PINT_FOR_EACH_NLON(PINT_CASE)
#undef PINT_CASE
        default:
          set_error("no ring FFT for nlon=%d", p.nlon);
          return PINT_E_INVAL;
      }
      PINT_HIP(hipGetLastError());
    }
    pint_status st = legendre_anal(p, nb, 1, s);
    if (st != PINT_OK) return st;
    st = scalar_post(p, spec + (size_t)b0 * p.ncoef * 2, nb, s);
    if (st != PINT_OK) return st;
  }
  return PINT_OK;
}

}  // namespace pint
