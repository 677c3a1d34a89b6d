// Latitude-ring kernels: the FFT half of the spectral transform (Sec. 2.2)
// fused with the pointwise nonlinear terms (Sec. 2.1, A-grid pseudospectral
// evaluation).  One workgroup per (latitude j, state b); the ring lives in LDS.
//
// Two FFT forms live here:
//  * the tendency kernel (k_ring_tendency, the hot one) carries every real
//    field of a ring as a half-length complex signal z[n] = x[2n] + i x[2n+1]
//    and transforms it in place in LDS, decimation in frequency for the
//    inverse transforms and decimation in time for the forward ones, so that
//    the pointwise products work on digit-reversed points (described above
//    the kernel);
//  * the scalar-transform, diagnostic and semi-Lagrangian ring kernels pair
//    two real signals in one complex FFT (x + i y), a mixed-radix
//    (4, 2, 3, 5) Stockham transform in one LDS buffer per signal pair:
//    each pass loads its butterflies' operands into registers, synchronises,
//    then writes the butterfly outputs.
#include <type_traits>

#include "pint_internal.h"

namespace pint {

// Complex arithmetic on double2 (FP64 path) and float2 (FP32 Legendre mode).
template <typename C>
struct CxTraits;
template <>
struct CxTraits<double2> {
  typedef double R;
};
template <>
struct CxTraits<float2> {
  typedef float R;
};
template <typename C>
using RealOf = typename CxTraits<C>::R;
template <typename T>
struct CxOf;
template <>
struct CxOf<double> {
  typedef double2 C;
};
template <>
struct CxOf<float> {
  typedef float2 C;
};

template <typename C>
__device__ inline C mkc(RealOf<C> x, RealOf<C> y) {
  C r;
  r.x = x;
  r.y = y;
  return r;
}
template <typename C>
__device__ inline C c_add(C a, C b) { return mkc<C>(a.x + b.x, a.y + b.y); }
template <typename C>
__device__ inline C c_sub(C a, C b) { return mkc<C>(a.x - b.x, a.y - b.y); }
template <typename C>
__device__ inline C c_scl(C a, RealOf<C> s) { return mkc<C>(a.x * s, a.y * s); }
// multiply by sign * i
template <typename C>
__device__ inline C c_si(C a, RealOf<C> sign) { return mkc<C>(-sign * a.y, sign * a.x); }
template <typename C>
__device__ inline C c_mul(C x, C y) {
  return mkc<C>(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}

template <int R1, int R2, typename C>
__device__ inline void dft_split(C* v, RealOf<C> sign);

// In-register DFT of size R: y_k = sum_r v_r exp(sign 2 pi i r k / R).
template <int R, typename C>
__device__ inline void dft(C* v, RealOf<C> sign) {
  using T = RealOf<C>;
  if constexpr (R == 2) {
    const C a = v[0], b = v[1];
    v[0] = c_add(a, b);
    v[1] = c_sub(a, b);
  } else if constexpr (R == 3) {
    const T h = T(0.86602540378443864676);   // sin(2 pi / 3)
    const C t = c_add(v[1], v[2]);
    const C d = c_sub(v[1], v[2]);
    const C base = c_sub(v[0], c_scl(t, T(0.5)));
    const C rot = c_si(c_scl(d, h), sign);
    v[0] = c_add(v[0], t);
    v[1] = c_add(base, rot);
    v[2] = c_sub(base, rot);
  } else if constexpr (R == 4) {
    const C s02 = c_add(v[0], v[2]), d02 = c_sub(v[0], v[2]);
    const C s13 = c_add(v[1], v[3]), d13 = c_si(c_sub(v[1], v[3]), sign);
    v[0] = c_add(s02, s13);
    v[2] = c_sub(s02, s13);
    v[1] = c_add(d02, d13);
    v[3] = c_sub(d02, d13);
  } else if constexpr (R == 5) {
    const T c1 = T(0.30901699437494742410), c2 = T(-0.80901699437494742410);   // cos 2pi/5, 4pi/5
    const T s1 = T(0.95105651629515357212), s2 = T(0.58778525229247312917);    // sin 2pi/5, 4pi/5
    const C a1 = c_add(v[1], v[4]), a2 = c_add(v[2], v[3]);
    const C b1 = c_sub(v[1], v[4]), b2 = c_sub(v[2], v[3]);
    const C y0 = c_add(v[0], c_add(a1, a2));
    const C r1 = c_add(v[0], c_add(c_scl(a1, c1), c_scl(a2, c2)));
    const C r2 = c_add(v[0], c_add(c_scl(a1, c2), c_scl(a2, c1)));
    const C i1 = c_si(c_add(c_scl(b1, s1), c_scl(b2, s2)), sign);
    const C i2 = c_si(c_sub(c_scl(b1, s2), c_scl(b2, s1)), sign);
    v[0] = y0;
    v[1] = c_add(r1, i1);
    v[4] = c_sub(r1, i1);
    v[2] = c_add(r2, i2);
    v[3] = c_sub(r2, i2);
  } else if constexpr (R == 6) {
    C a[3] = {v[0], v[2], v[4]};
    C b[3] = {v[1], v[3], v[5]};
    dft<3>(a, sign);
    dft<3>(b, sign);
    const T h = T(0.86602540378443864676) * sign;   // sign * sin(pi/3)
    // b_k *= exp(sign 2 pi i k / 6)
    const C b1 = mkc<C>(T(0.5) * b[1].x - h * b[1].y, h * b[1].x + T(0.5) * b[1].y);
    const C b2 = mkc<C>(T(-0.5) * b[2].x - h * b[2].y, h * b[2].x - T(0.5) * b[2].y);
    v[0] = c_add(a[0], b[0]);
    v[3] = c_sub(a[0], b[0]);
    v[1] = c_add(a[1], b1);
    v[4] = c_sub(a[1], b1);
    v[2] = c_add(a[2], b2);
    v[5] = c_sub(a[2], b2);
  } else if constexpr (R == 8) {
    dft_split<2, 4>(v, sign);
  } else {
    static_assert(R == 16, "radix");
    dft_split<4, 4>(v, sign);
  }
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
template <int R, int T, typename C>
__device__ inline C mul_w(C v, RealOf<C> sign) {
  using F = RealOf<C>;
  constexpr int t = (T * (16 / R)) % 16;
  if constexpr (t == 0) {
    return v;
  } else if constexpr (t == 4) {
    return c_si(v, sign);
  } else if constexpr (t == 8) {
    return mkc<C>(-v.x, -v.y);
  } else if constexpr (t == 12) {
    return c_si(v, -sign);
  } else {
    constexpr C2 w = w16(t);
    const F wc = F(w.c), ws = sign * F(w.s);
    return mkc<C>(v.x * wc - v.y * ws, v.x * ws + v.y * wc);
  }
}

// In-register DFT of size R1 * R2 by one Cooley-Tukey split: inner DFTs of
// size R2 over v[n1 + R1 n2], twiddles exp(sign 2 pi i n1 k2 / R), outer DFTs
// of size R1; output index k2 + R2 k1.
template <int R1, int R2, int N1 = 0, typename C>
__device__ inline void split_inner(C (&u)[R1][R2], const C* v, RealOf<C> sign) {
  if constexpr (N1 < R1) {
    C t[R2];
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) t[n2] = v[N1 + R1 * n2];
    dft<R2>(t, sign);
#pragma unroll
    for (int k2 = 0; k2 < R2; ++k2) u[N1][k2] = t[k2];
    split_inner<R1, R2, N1 + 1>(u, v, sign);
  }
}

template <int R1, int R2, int N1 = 1, int K2 = 1, typename C>
__device__ inline void split_twiddle(C (&u)[R1][R2], RealOf<C> sign) {
  if constexpr (N1 < R1) {
    if constexpr (K2 < R2) {
      u[N1][K2] = mul_w<R1 * R2, N1 * K2>(u[N1][K2], sign);
      split_twiddle<R1, R2, N1, K2 + 1>(u, sign);
    } else {
      split_twiddle<R1, R2, N1 + 1, 1>(u, sign);
    }
  }
}

template <int R1, int R2, typename C>
__device__ inline void dft_split(C* v, RealOf<C> sign) {
  C u[R1][R2];
  split_inner<R1, R2>(u, v, sign);
  split_twiddle<R1, R2>(u, sign);
#pragma unroll
  for (int k2 = 0; k2 < R2; ++k2) {
    C t[R1];
#pragma unroll
    for (int n1 = 0; n1 < R1; ++n1) t[n1] = u[n1][k2];
    dft<R1>(t, sign);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) v[k2 + R2 * k1] = t[k1];
  }
}

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
// Tendency ring kernel (one workgroup of kHThreads per latitude ring and
// state).  Every real grid field x of the ring (nlon = N = 2H points) is
// carried as the half-length complex signal z[n] = x[2n] + i x[2n+1]:
//   synthesis: Z[k] = (X_k + conj X_{H-k}) + i e^{2 pi i k/N} (X_k - conj X_{H-k}),
//              z = inverse FFT_H(Z)  (X_m = 0 for m > M, X_0 real);
//   analysis:  Z = FFT_H(z),  X_k = 1/2 [(Z_k + conj Z_{H-k})
//                                  - i e^{-2 pi i k/N} (Z_k - conj Z_{H-k})].
// Each field owns its transform (no pairing of unrelated fields, so no field
// inherits the rounding of a larger one).  The inverse transforms are in-place
// decimation in frequency (natural order in, digit-reversed out) and the
// forward ones decimation in time with the stage order reversed
// (digit-reversed in, natural out): the pointwise products work on the
// digit-reversed points directly, and every stage needs one barrier only.
//
// Fields (Sec. 2.1, advective form of N_A plus N_R), c^2 = 1 - mu_j^2:
//   N_Phi = -(U dPhi'/dlambda + V G) / (a c^2) - Phi' delta
//   K = (U^2 + V^2) / (2 c^2),  A = xi U / c^2,  B = xi V / c^2,
// each scaled by w_j / nlon, whose transforms m = 0..M go to
// G[m][j][(b*4 + f)*2] with f = (N_Phi, K, A, B).  The seven synthesised
// fields are transformed in two groups through a four-signal LDS buffer:
// (xi, delta, Phi'), whose xi and Phi' delta stay in registers, then
// (U, V, G, dPhi'/dlambda).
// ---------------------------------------------------------------------------
// Workgroup size: 128 threads (two waves) for batched launches, 256 (four
// waves, one signal each) for one or two states, where the ring's own
// latency sets the kernel time.  The arithmetic of a ring is the same for
// both (batch invariance).
constexpr int kHThreads = 128;
constexpr int kHThreadsSmall = 256;


constexpr int ilog2c(int n) {
  int c = 0;
  while (n > 1) { n >>= 1; ++c; }
  return c;
}
// Radix plan of a half-length transform of H points: stage 0 (span H) has
// radix 6, 5 or 8 (H divisible by 3, by 5, or a power of two); the remaining
// power of two 2^k goes in radix-8 stages, with one radix-4 stage when
// k = 2 (mod 3) and two when k = 1 (mod 3) -- as few passes over the LDS
// signals as the in-register butterflies allow.  The forward transform ends
// with stage 0 at stride H / R_0, which is even for every supported ring, so
// its butterflies j and S - j pair up as Z_k, Z_{H-k}.
constexpr int hplan_first(int H) { return H % 3 == 0 ? 6 : (H % 5 == 0 ? 5 : 8); }
constexpr int hplan_restlog(int H) { return ilog2c(H / hplan_first(H)); }
constexpr int hplan_n4(int H) {
  return hplan_restlog(H) % 3 == 0 ? 0 : (hplan_restlog(H) % 3 == 2 ? 1 : 2);
}
constexpr int hplan_n8(int H) { return (hplan_restlog(H) - 2 * hplan_n4(H)) / 3; }
constexpr int hplan_npass(int H) { return 1 + hplan_n8(H) + hplan_n4(H); }
constexpr int hplan_radix(int H, int i) {
  return i == 0 ? hplan_first(H) : (i <= hplan_n8(H) ? 8 : 4);
}
constexpr int hplan_span(int H, int i) {
  int L = H;
  for (int k = 0; k < i; ++k) L /= hplan_radix(H, k);
  return L;
}
constexpr bool hplan_ok(int H) {
  return hplan_span(H, hplan_npass(H)) == 1 && (H / hplan_first(H)) % 2 == 0;
}

// LDS layout of the half-length signals: signal s, point i at s*SP + i + i/16.
// SP is the padded signal length raised to 4 (mod 8) points, so that the
// four signals' points i start in different bank groups (record-wise staging
// touches all four signals at one i).
template <int H>
struct HRing {
  static constexpr int SP0 = H + H / 16;
  static constexpr int SP = SP0 + (12 - SP0 % 8) % 8;
  static_assert(SP % 8 == 4 && SP >= SP0, "signal stride");
  __device__ static inline int at(int s, int i) { return s * SP + i + (i >> 4); }
};

// exp(SGN 2 pi i t / N) from the table tw[t] = exp(-2 pi i t / N).
template <int SGN, typename C>
__device__ inline C twid(const C* __restrict__ tw, int t) {
  C w = tw[t];
  if constexpr (SGN > 0) w.y = -w.y;
  return w;
}

// Orders one wave's LDS accesses across this point: the LDS executes a
// wave's instructions in order, so only the compiler must not move them.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// One in-place stage (span L, radix R, stride S = L/R) over NSIG signals.
// DIF: butterfly, then twiddles W_L^{j r}; DIT: twiddles, then butterfly.
// Each wave of the workgroup owns whole signals (wave w: signals
// [w NW, (w+1) NW)), so the stages of a transform need no workgroup barrier:
// a wave only reads points it wrote itself.  The caller separates the
// transform from phases that mix signals with a workgroup barrier.
template <int H, int NSIG, int R, int L, bool kDif, int SGN, int NT, typename C>
__device__ inline void ip_stage(C* buf, const C* __restrict__ tw, int tid) {
  constexpr int S = L / R;
  constexpr int NBS = H / R;
  constexpr int NWAVE = NT / 64;
  constexpr int NW = (NSIG + NWAVE - 1) / NWAVE;     // signals per wave
  constexpr int TOTW = NW * NBS;
  constexpr int NIT = (TOTW + 63) / 64;
  constexpr int TWS = 2 * H / L;        // table step per unit of j r
  using Lay = HRing<H>;
  const int wave = tid >> 6, lane = tid & 63;
  const int s0 = wave * NW;
  const int tot = (NSIG - s0 < NW ? NSIG - s0 : NW) * NBS;   // this wave's butterflies
#pragma unroll
  for (int it = 0; it < NIT; ++it) {
    const int id = lane + it * 64;
    if (id < tot) {
      const int sw = id / NBS, rem = id - sw * NBS;
      const int sig = s0 + sw;
      // lanes run along j for wide strides and along the blocks for strides
      // <= 4, so that the lanes of one LDS access hit distinct banks
      int blk, j;
      if constexpr (S <= 4) {
        constexpr int NBLK = H / L;
        j = rem / NBLK;
        blk = rem - j * NBLK;
      } else {
        blk = rem / S;
        j = rem - blk * S;
      }
      const int base = blk * L + j;
      C v[R];
#pragma unroll
      for (int r = 0; r < R; ++r) v[r] = buf[Lay::at(sig, base + r * S)];
      // twiddles W^{j r}, r = 1..R-1: W from the table, its powers as
      // complex products (a few roundings each, far below the tolerances)
      C w[R];
      if constexpr (S > 1) {
        w[1] = twid<SGN>(tw, j * TWS);
        if constexpr (R > 2) w[2] = c_mul(w[1], w[1]);
#pragma unroll
        for (int r = 3; r < R; ++r) w[r] = c_mul(w[r - 2], w[2]);
      }
      if constexpr (!kDif && S > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = c_mul(v[r], w[r]);
      }
      dft<R>(v, RealOf<C>(SGN));
      if constexpr (kDif && S > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[r] = c_mul(v[r], w[r]);
      }
#pragma unroll
      for (int r = 0; r < R; ++r) buf[Lay::at(sig, base + r * S)] = v[r];
    }
  }
  wave_lds_sync();
}

template <int H, int NSIG, int SGN, int I, int NT, typename C>
__device__ inline void dif_stages(C* buf, const C* __restrict__ tw, int tid) {
  if constexpr (I < hplan_npass(H)) {
    ip_stage<H, NSIG, hplan_radix(H, I), hplan_span(H, I), true, SGN, NT>(buf, tw, tid);
    dif_stages<H, NSIG, SGN, I + 1, NT>(buf, tw, tid);
  }
}

// DIT stages I, I-1, ..., 1 (stage 0 is done by the caller).
template <int H, int NSIG, int SGN, int I, int NT, typename C>
__device__ inline void dit_stages(C* buf, const C* __restrict__ tw, int tid) {
  if constexpr (I >= 1) {
    ip_stage<H, NSIG, hplan_radix(H, I), hplan_span(H, I), false, SGN, NT>(buf, tw, tid);
    dit_stages<H, NSIG, SGN, I - 1, NT>(buf, tw, tid);
  }
}

// Z = (X1 + conj X2) + i w (X1 - conj X2)
template <typename C>
__device__ inline C hpre(C X1, C X2, C w) {
  const C d = mkc<C>(X1.x - X2.x, X1.y + X2.y);
  const C wd = c_mul(w, d);
  return mkc<C>(X1.x + X2.x - wd.y, X1.y - X2.y + wd.x);
}

// X = 1/2 [(Za + conj Zb) - i w (Za - conj Zb)]
template <typename C>
__device__ inline C hpost(C Za, C Zb, C w) {
  using T = RealOf<C>;
  const C d = mkc<C>(Za.x - Zb.x, Za.y + Zb.y);
  const C wd = c_mul(w, d);
  return mkc<C>(T(0.5) * (Za.x + Zb.x + wd.y), T(0.5) * (Za.y - Zb.y - wd.x));
}

template <int N, typename T, int NT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(3))) void k_ring_tendency(
    const T* __restrict__ F, T* __restrict__ Gout, const double* __restrict__ c2,
    const double* __restrict__ w, const typename CxOf<T>::C* __restrict__ tw, int M, int nlat,
    int nlat2, int B, double a) {
  using C = typename CxOf<T>::C;
  constexpr int H = N / 2;
  static_assert(hplan_ok(H), "no half-length plan for this ring");
  constexpr int NPW = (H + NT - 1) / NT;   // pointwise points per thread
  using Lay = HRing<H>;
  extern __shared__ __align__(16) unsigned char ring_lds[];
  C* zb = reinterpret_cast<C*>(ring_lds);
  // logical block = ((jn * B) + b) * 2 + hemisphere: the rings of one state
  // run back to back on one XCD
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int hemi = lb & 1, rb = lb >> 1;
  const int jn = rb / B, b = rb - jn * B;
  const int j = hemi ? nlat - 1 - jn : jn;
  const int ncs = 12 * B;
  const int tid = threadIdx.x;
  // Fourier coefficients of this ring: record (m, j, b) holds the six
  // synthesised fields contiguously
  const T* frow = F + (size_t)j * ncs + b * 12;
  const size_t fstride = fourier_pitch<T>(nlat, ncs);   // between m and m + 1
  // Stage NS fields' coefficients in LDS, slot s at point m for m <= M.
  // Lanes run over the fields of a record (a few cache lines per wave
  // access); a thread's loads are all issued before its first LDS store.
  auto stage_in = [&](auto nsig, auto field_of) {
    constexpr int NS = decltype(nsig)::value;
    constexpr int NIT = (H * NS + NT - 1) / NT;   // M < H
    constexpr int CH = 6;                                        // loads in flight
    const int total = (M + 1) * NS;
#pragma unroll
    for (int c0 = 0; c0 < NIT; c0 += CH) {
      C v[CH];
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        const int it = (c0 + e) * NT + tid;
        const int m = it / NS, sl = it - m * NS;
        v[e] = (c0 + e < NIT && it < total)
                   ? *reinterpret_cast<const C*>(frow + m * fstride + 2 * field_of(sl))
                   : mkc<C>(T(0), T(0));
      }
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        const int it = (c0 + e) * NT + tid;
        if (c0 + e < NIT && it < total) {
          const int m = it / NS, sl = it - m * NS;
          zb[Lay::at(sl, m)] = v[e];
        }
      }
    }
    __syncthreads();
  };
  // Staged spectra of NS fields -> Z of the half-length signals, in place.
  // Thread q reads points q and H - q of each slot and writes Z at the same
  // two points, so no other thread touches them.  post(s, m, x) maps the
  // staged coefficient to the transformed one (i m x for a longitude
  // derivative).
  auto put = [&](auto nsig, auto post) {
    constexpr int NS = decltype(nsig)::value;
    constexpr int NQ = (H / 2 + NT) / NT;   // pairs (k, H-k) per thread
#pragma unroll
    for (int it = 0; it < NQ; ++it) {
      const int q = tid + it * NT;
      if (q <= H / 2) {
        const int k1 = q, k2 = H - q;
        const bool h1 = q <= M, h2 = q > 0 && k2 <= M;
        const C w1 = twid<1>(tw, k1);                // exp(2 pi i k1 / N)
        const C w2 = mkc<C>(-w1.x, w1.y);            // exp(2 pi i (H - k1) / N)
        C X1[NS], X2[NS];
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
          X1[sl] = h1 ? post(sl, k1, zb[Lay::at(sl, k1)]) : mkc<C>(T(0), T(0));
          X2[sl] = h2 ? post(sl, k2, zb[Lay::at(sl, k2)]) : mkc<C>(T(0), T(0));
          if (q == 0) X1[sl].y = T(0);               // a real field's mean
        }
#pragma unroll
        for (int sl = 0; sl < NS; ++sl) {
          zb[Lay::at(sl, k1)] = hpre(X1[sl], X2[sl], w1);
          if (q > 0 && k2 != k1) zb[Lay::at(sl, k2)] = hpre(X2[sl], X1[sl], w2);
        }
      }
    }
    __syncthreads();
  };
  auto ident = [](int, int, C x) -> C { return x; };

  const double ic2d = 1.0 / c2[j];
  const T ic2 = T(ic2d);
  const T ica = T(ic2d / a);
  const T sc = T(w[j] / N);
  // ---- group 1: xi, delta, Phi' -> keep xi and Phi' delta per point ----
  stage_in(std::integral_constant<int, 3>(), [](int sl) { return sl; });
  put(std::integral_constant<int, 3>(), ident);
  dif_stages<H, 3, 1, 0, NT>(zb, tw, tid);
  __syncthreads();
  C Xr[NPW], Dr[NPW];
#pragma unroll
  for (int t = 0; t < NPW; ++t) {
    const int p = tid + t * NT;
    if (H % NT == 0 || p < H) {
      const C xi = zb[Lay::at(0, p)], de = zb[Lay::at(1, p)], ph = zb[Lay::at(2, p)];
      Xr[t] = xi;
      Dr[t] = mkc<C>(ph.x * de.x, ph.y * de.y);
    }
  }
  __syncthreads();

  // ---- group 2: U, V, G, dPhi'/dlambda -> all four products ----
  // slots (U, V, G, Phi') from fields 4, 5, 3, 2; slot 3 becomes i m Phi'
  stage_in(std::integral_constant<int, 4>(), [](int sl) { return sl < 2 ? sl + 4 : 5 - sl; });
  put(std::integral_constant<int, 4>(), [](int sl, int m, C x) -> C {
    return sl == 3 ? mkc<C>(-T(m) * x.y, T(m) * x.x) : x;
  });
  dif_stages<H, 4, 1, 0, NT>(zb, tw, tid);
  __syncthreads();
#pragma unroll
  for (int t = 0; t < NPW; ++t) {
    const int p = tid + t * NT;
    if (H % NT == 0 || p < H) {
      const C U = zb[Lay::at(0, p)], V = zb[Lay::at(1, p)];
      const C G = zb[Lay::at(2, p)], L = zb[Lay::at(3, p)];
      const C xi = Xr[t], pd = Dr[t];
      zb[Lay::at(0, p)] = mkc<C>((-(U.x * L.x + V.x * G.x) * ica - pd.x) * sc,
                                 (-(U.y * L.y + V.y * G.y) * ica - pd.y) * sc);   // N_Phi
      zb[Lay::at(1, p)] = mkc<C>(xi.x * U.x * ic2 * sc, xi.y * U.y * ic2 * sc);   // A
      zb[Lay::at(2, p)] = mkc<C>(xi.x * V.x * ic2 * sc, xi.y * V.y * ic2 * sc);   // B
      zb[Lay::at(3, p)] = mkc<C>(T(0.5) * (U.x * U.x + V.x * V.x) * ic2 * sc,
                                 T(0.5) * (U.y * U.y + V.y * V.y) * ic2 * sc);    // K
    }
  }
  __syncthreads();

  // ---- forward transforms of (N_Phi, A, B, K) in slots 0..3 ----
  dit_stages<H, 4, -1, hplan_npass(H) - 1, NT>(zb, tw, tid);
  __syncthreads();
  // last stage (span H) with the pairing k <-> H - k and the unpacking,
  // written back in place (a thread writes only the points it read)
  constexpr int R1 = hplan_first(H), S1 = H / R1, UPS = S1 / 2;
  constexpr int TOTU = 4 * UPS;
  const int ncg = 8 * B;
  for (int u = tid; u < TOTU; u += NT) {
    const int sig = u / UPS, uu = u - sig * UPS;
    const int ja = uu, jb = uu == 0 ? S1 / 2 : S1 - uu;
    C za[R1], zc[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      za[r] = zb[Lay::at(sig, ja + r * S1)];
      zc[r] = zb[Lay::at(sig, jb + r * S1)];
    }
    C wa[R1], wc[R1];                                // W^{j r}: W loaded
    wa[1] = twid<-1>(tw, ja * 2);
    wc[1] = twid<-1>(tw, jb * 2);
    if constexpr (R1 > 2) {
      wa[2] = c_mul(wa[1], wa[1]);
      wc[2] = c_mul(wc[1], wc[1]);
    }
#pragma unroll
    for (int r = 3; r < R1; ++r) {
      wa[r] = c_mul(wa[r - 2], wa[2]);
      wc[r] = c_mul(wc[r - 2], wc[2]);
    }
#pragma unroll
    for (int r = 1; r < R1; ++r) {
      za[r] = c_mul(za[r], wa[r]);
      zc[r] = c_mul(zc[r], wc[r]);
    }
    dft<R1>(za, T(-1));
    dft<R1>(zc, T(-1));
    C xa[R1], xc[R1];
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int ka = ja + r * S1, kc = jb + r * S1;
      // partners Z_{H-k}
      const C pa = uu == 0 ? za[(R1 - r) % R1] : zc[R1 - 1 - r];
      const C pc = uu == 0 ? zc[R1 - 1 - r] : za[R1 - 1 - r];
      xa[r] = hpost(za[r], pa, tw[ka]);
      xc[r] = hpost(zc[r], pc, tw[kc]);
    }
#pragma unroll
    for (int r = 0; r < R1; ++r) {
      const int ka = ja + r * S1, kc = jb + r * S1;
      if (ka <= M) zb[Lay::at(sig, ka)] = xa[r];
      if (kc <= M) zb[Lay::at(sig, kc)] = xc[r];
    }
  }
  __syncthreads();
  // results (N_Phi, K, A, B) = slots (0, 3, 1, 2) to G, lanes over the four
  // fields of a record
  T* grow = Gout + (size_t)j * ncg + b * 8;
  const size_t gstride = fourier_pitch<T>(nlat, ncg);
  for (int it = tid; it < (M + 1) * 4; it += NT) {
    const int m = it >> 2, f = it & 3;
    const int sl = f == 0 ? 0 : (f == 1 ? 3 : f - 1);
    *reinterpret_cast<C*>(grow + m * gstride + 2 * f) = zb[Lay::at(sl, m)];
  }
}

// ---------------------------------------------------------------------------
// Scalar rings for the public transforms (two states per workgroup).
// synthesis: Fourier rows F[m][j][b] (nf = 1) -> grid[b][j][k]
// analysis:  grid[b][j][k] -> G[m][j][b*2] scaled by w_j / nlon
// ---------------------------------------------------------------------------
// SQ: instead of storing the grid, sum the squares of the pair over the
// ring into grid[pair][latitude][2] (physical-space L2 norms).
template <int N, bool SQ>
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
  const int ncs = 2 * B;
  auto fourier = [&](int m, double2* x, double2* y) {
    const double2* f = reinterpret_cast<const double2*>(F + m * fourier_pitch<double>(nlat, ncs) +
                                                        (size_t)j * ncs);
    *x = f[b0];
    *y = two ? f[b0 + 1] : make_double2(0.0, 0.0);
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
  if constexpr (SQ) {
    double acc[2] = {0.0, 0.0};
    for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
      const double2 z = zb[L::at(0, k)];
      const double y = z.y * isc;
      acc[0] += z.x * z.x;
      acc[1] += y * y;
    }
    block_sum<2>(acc, red, threadIdx.x);
    // a signal whose Fourier coefficients on this ring are all zero is zero
    // on the ring: drop the rounding its partner leaks into it
    if (threadIdx.x == 0) {
      grid[((size_t)blockIdx.y * nlat + j) * 2] = nrm[0] > 0.0 ? acc[0] : 0.0;
      grid[((size_t)blockIdx.y * nlat + j) * 2 + 1] = two && nrm[1] > 0.0 ? acc[1] : 0.0;
    }
  } else {
    for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
      const double2 z = zb[L::at(0, k)];
      grid[((size_t)b0 * nlat + j) * nlon + k] = z.x;
      if (two) grid[((size_t)(b0 + 1) * nlat + j) * nlon + k] = z.y * isc;
    }
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
    double2* g = reinterpret_cast<double2*>(Gout + m * fourier_pitch<double>(nlat, ncg) +
                                              (size_t)j * ncg);
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

// Dynamic LDS of the tendency ring kernel: 4 half-length signals (complex
// FP64, or FP32 in the mixed-precision mode).
size_t ring_lds_bytes(int nlon, int prec) {
  const size_t cx = prec != PINT_FP64 ? sizeof(float2) : sizeof(double2);
  switch (nlon) {
#define PINT_CASE(n) \
  case n:            \
    return (size_t)4 * HRing<n / 2>::SP * cx;
    PINT_FOR_EACH_NLON(PINT_CASE)
#undef PINT_CASE
    default:
      return 0;
  }
}

// Allow the tendency ring kernels their dynamic LDS.
pint_status ring_prepare(int nlon) {
  switch (nlon) {
#define PINT_CASE(n)                                                                          \
  case n:                                                                                     \
    PINT_HIP(hipFuncSetAttribute((const void*)k_ring_tendency<n, double, kHThreads>,          \
                                 hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                                 (int)ring_lds_bytes(n, PINT_FP64)));                         \
    PINT_HIP(hipFuncSetAttribute((const void*)k_ring_tendency<n, float, kHThreads>,           \
                                 hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                                 (int)ring_lds_bytes(n, PINT_LEG_FP32)));                     \
    PINT_HIP(hipFuncSetAttribute((const void*)k_ring_tendency<n, double, kHThreadsSmall>,     \
                                 hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                                 (int)ring_lds_bytes(n, PINT_FP64)));                         \
    PINT_HIP(hipFuncSetAttribute((const void*)k_ring_tendency<n, float, kHThreadsSmall>,      \
                                 hipFuncAttributeMaxDynamicSharedMemorySize,                  \
                                 (int)ring_lds_bytes(n, PINT_LEG_FP32)));                     \
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
  const bool f32 = p.prec != PINT_FP64;
  // workgroup size: 256 threads (one wave per signal) by default for one or
  // two states, 128 for more; the plan's tuned variant may swap them (the
  // arithmetic of a ring is the same in both)
  const bool small = (B <= 2) != (p.ring_variant[B <= 2 ? 0 : 1] == 1);
  switch (p.nlon) {
#define PINT_LAUNCH(n, T, NT, f, g, tw)                                                      \
  hipLaunchKernelGGL((k_ring_tendency<n, T, NT>), dim3(p.nlat * B), dim3(NT),                \
                     ring_lds_bytes(n, p.prec), s, f, g, p.c2, p.w, tw, p.M, p.nlat, p.nlat2, B, \
                     p.a)
#define PINT_CASE(n)                                                                         \
  case n:                                                                                    \
    if (f32 && small)                                                                        \
      PINT_LAUNCH(n, float, kHThreadsSmall, reinterpret_cast<const float*>(p.F),             \
                  reinterpret_cast<float*>(p.G), p.twid32);                                  \
    else if (f32)                                                                            \
      PINT_LAUNCH(n, float, kHThreads, reinterpret_cast<const float*>(p.F),                  \
                  reinterpret_cast<float*>(p.G), p.twid32);                                  \
    else if (small)                                                                          \
      PINT_LAUNCH(n, double, kHThreadsSmall, p.F, p.G, p.twid);                             \
    else                                                                                     \
      PINT_LAUNCH(n, double, kHThreads, p.F, p.G, p.twid);                                  \
    break;
    PINT_FOR_EACH_NLON(PINT_CASE)
#undef PINT_CASE
#undef PINT_LAUNCH
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
    st = legendre_synth(p, nb, 1, PINT_FP64, s);
    if (st != PINT_OK) return st;
    {
      ProfScope ps(p, PK_SRING, nb, s);
      double* gout = grid + (size_t)b0 * p.nlat * p.nlon;
      switch (p.nlon) {
#define PINT_CASE(n)                                                                             \
  case n:                                                                                        \
    hipLaunchKernelGGL((k_ring_synth<n, false>), dim3(p.nlat, (nb + 1) / 2), dim3(kRingThreads), \
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

pint_status ring_sumsq(Plan& p, int nspec, double* part, hipStream_t s) {
  ProfScope ps(p, PK_SRING, nspec, s);
  switch (p.nlon) {
#define PINT_CASE(n)                                                                             \
  case n:                                                                                        \
    hipLaunchKernelGGL((k_ring_synth<n, true>), dim3(p.nlat, (nspec + 1) / 2),                   \
                       dim3(kRingThreads), (size_t)RingLds<n>::SP * sizeof(double2), s, p.F,     \
                       part, p.twid, p.M, p.nlat, p.nlat2, nspec);                               \
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
    pint_status st = legendre_anal(p, nb, 1, PINT_FP64, s);
    if (st != PINT_OK) return st;
    st = scalar_post(p, spec + (size_t)b0 * p.ncoef * 2, nb, s);
    if (st != PINT_OK) return st;
  }
  return PINT_OK;
}


// ---------------------------------------------------------------------------
// Semi-Lagrangian step (Sec. 2.3.2): rings between the synthesised Fourier
// coefficients and grid-point fields.
// k_ring_sl_grid: the six synthesised fields of state b (record layout of the
//   tendency path) -> grid[b][o][j][k] for o = delta, Phi', G = (1-mu^2)
//   dPhi'/dmu, dPhi'/dlambda, U = u cos(lat), V = v cos(lat); three pairs of
//   real signals through one complex FFT each.
// k_ring_sl_anal: grid[b][g][j][k] for g = (R_Phi, A, B) -> ring-output
//   records (N_Phi <- R_Phi, K <- 0, A, B) scaled by w_j / nlon, the layout
//   the analysis GEMM and the tendency assembly read.
// ---------------------------------------------------------------------------
template <int N>
__global__ __launch_bounds__(kRingThreads) void k_ring_sl_grid(const double* __restrict__ F,
                                                               double* __restrict__ grid,
                                                               const double2* __restrict__ tw,
                                                               int M, int nlat, int Bt) {
  constexpr int nlon = N;
  using L = RingLds<N>;
  extern __shared__ double2 zb[];
  __shared__ double red[kRingWaves * 6];
  const int j = blockIdx.x, b = blockIdx.y;
  const int ncs = 12 * Bt;
  const size_t fstride = fourier_pitch<double>(nlat, ncs);
  const double* rec = F + (size_t)j * ncs + (size_t)b * 12;
  // pair s: (X, Y) = (delta, Phi'), (G, i m Phi'), (U, V)
  auto coef = [&](int m, int s, double2* X, double2* Y) {
    const double* r = rec + m * fstride;
    if (s == 0) {
      *X = *reinterpret_cast<const double2*>(r + 2);
      *Y = *reinterpret_cast<const double2*>(r + 4);
    } else if (s == 1) {
      *X = *reinterpret_cast<const double2*>(r + 6);
      const double2 ph = *reinterpret_cast<const double2*>(r + 4);
      *Y = make_double2(-m * ph.y, m * ph.x);
    } else {
      *X = *reinterpret_cast<const double2*>(r + 8);
      *Y = *reinterpret_cast<const double2*>(r + 10);
    }
  };
  double nrm[6] = {0, 0, 0, 0, 0, 0};
  for (int m = threadIdx.x; m <= M; m += kRingThreads) {
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      double2 x, y;
      coef(m, s, &x, &y);
      nrm[2 * s] += x.x * x.x + x.y * x.y;
      nrm[2 * s + 1] += y.x * y.x + y.y * y.y;
    }
  }
  block_sum<6>(nrm, red, threadIdx.x);
  double sc[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) sc[s] = pair_scale(nrm[2 * s], nrm[2 * s + 1]);
  for (int i = threadIdx.x; i < 3 * L::SP; i += kRingThreads) zb[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int m = threadIdx.x; m <= M; m += kRingThreads) {
#pragma unroll
    for (int s = 0; s < 3; ++s) {
      double2 x, y;
      coef(m, s, &x, &y);
      put_pair<N>(zb, s, m, x, c_scl(y, sc[s]));
    }
  }
  __syncthreads();
  fft_lds<N, 3>(zb, 1.0, tw, threadIdx.x);
  const size_t plane = (size_t)nlat * nlon;
  double* out = grid + (size_t)b * 6 * plane + (size_t)j * nlon;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    const double isc = 1.0 / sc[s];
    for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
      const double2 z = zb[L::at(s, k)];
      out[(2 * s) * plane + k] = z.x;
      out[(2 * s + 1) * plane + k] = z.y * isc;
    }
  }
}

template <int N>
__global__ __launch_bounds__(kRingThreads) void k_ring_sl_anal(const double* __restrict__ grid,
                                                               double* __restrict__ Gout,
                                                               const double* __restrict__ w,
                                                               const double2* __restrict__ tw,
                                                               int M, int nlat, int B) {
  constexpr int nlon = N;
  using L = RingLds<N>;
  extern __shared__ double2 zb[];
  __shared__ double red[kRingWaves * 2];
  const int j = blockIdx.x, b = blockIdx.y;
  const size_t plane = (size_t)nlat * nlon;
  const double* g = grid + (size_t)b * 3 * plane + (size_t)j * nlon;
  const double sc = w[j] / nlon;
  double nrm[2] = {0, 0};
  for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
    const double x = g[k], y = g[plane + k];
    nrm[0] += x * x;
    nrm[1] += y * y;
  }
  block_sum<2>(nrm, red, threadIdx.x);
  const double s0 = pair_scale(nrm[0], nrm[1]);
  for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
    zb[L::at(0, k)] = make_double2(g[k] * sc, g[plane + k] * s0 * sc);
    zb[L::at(1, k)] = make_double2(g[2 * plane + k] * sc, 0.0);
  }
  __syncthreads();
  fft_lds<N, 2>(zb, -1.0, tw, threadIdx.x);
  const int ncg = 8 * B;
  const double is0 = 1.0 / s0;
  for (int m = threadIdx.x; m <= M; m += kRingThreads) {
    double2 X, Y, Z, D;
    get_pair<N>(zb, 0, m, &X, &Y);
    get_pair<N>(zb, 1, m, &Z, &D);
    double2* r = reinterpret_cast<double2*>(Gout + m * fourier_pitch<double>(nlat, ncg) +
                                            (size_t)j * ncg + (size_t)b * 8);
    r[0] = X;
    r[1] = make_double2(0.0, 0.0);
    r[2] = c_scl(Y, is0);
    r[3] = Z;
  }
}

pint_status ring_sl_grid(Plan& p, double* grid, int Bt, hipStream_t s) {
  ProfScope ps(p, PK_SRING, Bt, s);
  switch (p.nlon) {
#define PINT_CASE(n)                                                                            \
  case n:                                                                                       \
    hipLaunchKernelGGL(k_ring_sl_grid<n>, dim3(p.nlat, Bt), dim3(kRingThreads),                 \
                       (size_t)3 * RingLds<n>::SP * sizeof(double2), s, p.F, grid, p.twid, p.M, \
                       p.nlat, Bt);                                                             \
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

pint_status ring_sl_anal(Plan& p, const double* grid, int B, hipStream_t s) {
  ProfScope ps(p, PK_SRING, B, s);
  switch (p.nlon) {
#define PINT_CASE(n)                                                                            \
  case n:                                                                                       \
    hipLaunchKernelGGL(k_ring_sl_anal<n>, dim3(p.nlat, B), dim3(kRingThreads),                  \
                       (size_t)2 * RingLds<n>::SP * sizeof(double2), s, grid, p.G, p.w, p.twid, \
                       p.M, p.nlat, B);                                                         \
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

// Autotuner of the ring workgroup size: for each launch class, time both
// sizes at the class's batch on the plan's workspace and keep the faster
// (bitwise the same results).  Synchronises `s`.
pint_status tune_ring(Plan& p, const int (&states)[2], hipStream_t s) {
  hipEvent_t e0, e1;
  PINT_HIP(hipEventCreate(&e0));
  PINT_HIP(hipEventCreate(&e1));
  pint_status st = PINT_OK;
  for (int cls = 0; cls < 2 && st == PINT_OK; ++cls) {
    const int B = states[cls];
    if (B < 1 || B > p.max_batch || ((B <= 2) != (cls == 0))) continue;
    int best = 0;
    float best_ms = 0.0f;
    for (int v = 0; v < 2 && st == PINT_OK; ++v) {
      p.ring_variant[cls] = v;
      float ms = 0.0f;
      for (int rep = 0; rep < 4 && st == PINT_OK; ++rep) {   // first one warms up
        if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) st = PINT_E_HIP;
        if (st == PINT_OK) st = ring_tendency(p, B, s);
      }
      if (st == PINT_OK && (hipEventRecord(e1, s) != hipSuccess ||
                            hipEventSynchronize(e1) != hipSuccess ||
                            hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = PINT_E_HIP;
      if (st == PINT_OK && (v == 0 || ms < best_ms)) {
        best = v;
        best_ms = ms;
      }
    }
    p.ring_variant[cls] = best;
    p.ring_tuned_ms[cls] = best_ms / 3.0f;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == PINT_E_HIP) set_error("timing the ring kernel variants failed");
  return st;
}

}  // namespace pint
