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

struct RadixPlan {
  int n;
  int r[16];
};

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

// One Stockham pass of radix R over nsig signals of length N stored back to
// back in buf.  Ns = product of the radices of the earlier passes.
template <int R>
__device__ inline void fft_pass(double2* buf, int nsig, int N, int Ns, double sign,
                                const double2* __restrict__ tw) {
  const int nb = N / R;
  const int total = nsig * nb;
  double2 v[kFftMaxBf][R];
#pragma unroll
  for (int t = 0; t < kFftMaxBf; ++t) {
    const int id = threadIdx.x + t * kRingThreads;
    if (id < total) {
      const int sig = id / nb, j = id - sig * nb;
#pragma unroll
      for (int r = 0; r < R; ++r) v[t][r] = buf[sig * N + j + r * nb];
    }
  }
  __syncthreads();
  const int tstep = N / (Ns * R);
#pragma unroll
  for (int t = 0; t < kFftMaxBf; ++t) {
    const int id = threadIdx.x + t * kRingThreads;
    if (id < total) {
      const int sig = id / nb, j = id - sig * nb;
      const int k = j % Ns;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        double2 w = tw[r * k * tstep];          // exp(-2 pi i r k / (Ns R))
        if (sign > 0.0) w.y = -w.y;
        v[t][r] = cmul(v[t][r], w);
      }
      dft<R>(v[t], sign);
      const int o = sig * N + (j / Ns) * Ns * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[o + r * Ns] = v[t][r];
    }
  }
  __syncthreads();
}

// Complex FFT of nsig signals in LDS: sign -1 forward, +1 inverse (unnormalised).
__device__ void fft_lds(double2* buf, int nsig, int N, double sign, const RadixPlan& rp,
                        const double2* __restrict__ tw) {
  int Ns = 1;
  for (int i = 0; i < rp.n; ++i) {
    const int R = rp.r[i];
    if (R == 4)
      fft_pass<4>(buf, nsig, N, Ns, sign, tw);
    else if (R == 2)
      fft_pass<2>(buf, nsig, N, Ns, sign, tw);
    else if (R == 3)
      fft_pass<3>(buf, nsig, N, Ns, sign, tw);
    else
      fft_pass<5>(buf, nsig, N, Ns, sign, tw);
    Ns *= R;
  }
}

// Sum NV per-thread values over the workgroup (fixed order: wave shuffles,
// then the wave partials in LDS).  red must hold kRingWaves * NV doubles.
constexpr int kRingWaves = kRingThreads / 64;
template <int NV>
__device__ inline void block_sum(double (&v)[NV], double* red) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[i] += __shfl_xor(v[i], off);
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
__device__ inline void put_pair(double2* z, int N, int m, double2 X, double2 Y) {
  if (m == 0) {
    z[0] = make_double2(X.x, Y.x);
  } else {
    z[m] = make_double2(X.x - Y.y, X.y + Y.x);
    z[N - m] = make_double2(X.x + Y.y, Y.x - X.y);
  }
}

// Split Z = FFT(x + i y) of two real signals: X_m = (Z_m + conj Z_{-m}) / 2,
// Y_m = (Z_m - conj Z_{-m}) / (2i).
__device__ inline void get_pair(const double2* z, int N, int m, double2* X, double2* Y) {
  const double2 zp = z[m];
  const double2 zm = z[m == 0 ? 0 : N - m];
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
__global__ __launch_bounds__(kRingThreads) void k_ring_tendency(
    const double* __restrict__ F, double* __restrict__ Gout, const double* __restrict__ c2,
    const double* __restrict__ w, const double2* __restrict__ tw, RadixPlan rp, int M, int nlon,
    int nlat, int nlat2, int B, double a) {
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
  // field norms over the ring (Parseval, up to a common factor); when every
  // thread owns at most one m its Fourier values stay in registers
  const bool one = M < kRingThreads;
  double2 vc[7];
  double nrm[7] = {0, 0, 0, 0, 0, 0, 0};
  for (int m = tid; m <= M; m += kRingThreads) {
    double2 v[7];
    fourier(m, v);
#pragma unroll
    for (int f = 0; f < 7; ++f) {
      nrm[f] += v[f].x * v[f].x + v[f].y * v[f].y;
      vc[f] = v[f];
    }
  }
  block_sum<7>(nrm, red);
  // fields: 0 xi, 1 delta, 2 Phi', 3 G, 4 U, 5 V, 6 dPhi'/dlambda
  const double sUV = pair_scale(nrm[4], nrm[5]);
  const double sGL = pair_scale(nrm[3], nrm[6]);
  const double sXD = pair_scale(nrm[0], nrm[1]);
  for (int i = tid; i < 4 * nlon; i += kRingThreads) zb[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int m = tid; m <= M; m += kRingThreads) {
    double2 v[7];
    if (one) {
#pragma unroll
      for (int f = 0; f < 7; ++f) v[f] = vc[f];
    } else {
      fourier(m, v);
    }
    put_pair(zb, nlon, m, v[4], c_scl(v[5], sUV));              // U + i s V
    put_pair(zb + nlon, nlon, m, v[3], c_scl(v[6], sGL));       // G + i s dPhi'/dlambda
    put_pair(zb + 2 * nlon, nlon, m, v[0], c_scl(v[1], sXD));   // xi + i s delta
    put_pair(zb + 3 * nlon, nlon, m, v[2], make_double2(0.0, 0.0));  // Phi'
  }
  __syncthreads();
  fft_lds(zb, 4, nlon, 1.0, rp, tw);
  const double ic2 = 1.0 / c2[j];
  const double sc = w[j] / nlon;
  const double ia = 1.0 / a;
  const double iUV = 1.0 / sUV, iGL = 1.0 / sGL, iXD = 1.0 / sXD;
  double fn[4] = {0, 0, 0, 0};
  for (int k = tid; k < nlon; k += kRingThreads) {
    const double2 z1 = zb[k], z2 = zb[nlon + k], z3 = zb[2 * nlon + k], z4 = zb[3 * nlon + k];
    const double U = z1.x, V = z1.y * iUV, G = z2.x, phl = z2.y * iGL;
    const double xi = z3.x, de = z3.y * iXD, ph = z4.x;
    const double nphi = (-(U * phl + V * G) * ic2 * ia - ph * de) * sc;
    const double A = xi * U * ic2 * sc, Bv = xi * V * ic2 * sc;
    const double K = 0.5 * (U * U + V * V) * ic2 * sc;
    zb[k] = make_double2(nphi, K);
    zb[nlon + k] = make_double2(A, Bv);
    fn[0] += nphi * nphi;
    fn[1] += K * K;
    fn[2] += A * A;
    fn[3] += Bv * Bv;
  }
  block_sum<4>(fn, red);
  const double sNK = pair_scale(fn[0], fn[1]);
  const double sAB = pair_scale(fn[2], fn[3]);
  if (sNK != 1.0 || sAB != 1.0) {
    for (int k = tid; k < nlon; k += kRingThreads) {
      zb[k].y *= sNK;
      zb[nlon + k].y *= sAB;
    }
  }
  __syncthreads();
  fft_lds(zb, 2, nlon, -1.0, rp, tw);
  const int ncg = 8 * B;
  const double iNK = 1.0 / sNK, iAB = 1.0 / sAB;
  for (int m = tid; m <= M; m += kRingThreads) {
    double2 X0, Y0, X1, Y1;
    get_pair(zb, nlon, m, &X0, &Y0);
    get_pair(zb + nlon, nlon, m, &X1, &Y1);
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
__global__ __launch_bounds__(kRingThreads) void k_ring_synth(const double* __restrict__ F,
                                                             double* __restrict__ grid,
                                                             const double2* __restrict__ tw,
                                                             RadixPlan rp, int M, int nlon,
                                                             int nlat, int nlat2, int B) {
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
  block_sum<2>(nrm, red);
  const double sc = pair_scale(nrm[0], nrm[1]);
  for (int i = threadIdx.x; i < nlon; i += kRingThreads) zb[i] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int m = threadIdx.x; m <= M; m += kRingThreads) {
    double2 x, y;
    fourier(m, &x, &y);
    put_pair(zb, nlon, m, x, c_scl(y, sc));
  }
  __syncthreads();
  fft_lds(zb, 1, nlon, 1.0, rp, tw);
  const double isc = 1.0 / sc;
  for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
    grid[((size_t)b0 * nlat + j) * nlon + k] = zb[k].x;
    if (two) grid[((size_t)(b0 + 1) * nlat + j) * nlon + k] = zb[k].y * isc;
  }
}

__global__ __launch_bounds__(kRingThreads) void k_ring_anal(const double* __restrict__ grid,
                                                            double* __restrict__ Gout,
                                                            const double* __restrict__ w,
                                                            const double2* __restrict__ tw,
                                                            RadixPlan rp, int M, int nlon,
                                                            int nlat, int B) {
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
  block_sum<2>(nrm, red);
  const double s = pair_scale(nrm[0], nrm[1]);
  for (int k = threadIdx.x; k < nlon; k += kRingThreads) {
    const double x = grid[((size_t)b0 * nlat + j) * nlon + k];
    const double y = two ? grid[((size_t)(b0 + 1) * nlat + j) * nlon + k] : 0.0;
    zb[k] = make_double2(x * sc, y * s * sc);
  }
  __syncthreads();
  fft_lds(zb, 1, nlon, -1.0, rp, tw);
  const int ncg = 2 * B;
  const double is = 1.0 / s;
  for (int m = threadIdx.x; m <= M; m += kRingThreads) {
    double2 X, Y;
    get_pair(zb, nlon, m, &X, &Y);
    double2* g = reinterpret_cast<double2*>(Gout + ((size_t)m * nlat + j) * ncg);
    g[b0] = X;
    if (two) g[b0 + 1] = c_scl(Y, is);
  }
}

static RadixPlan rplan(const Plan& p) {
  RadixPlan rp;
  rp.n = p.nradix;
  for (int i = 0; i < 16; ++i) rp.r[i] = p.radix[i];
  return rp;
}

pint_status ring_tendency(Plan& p, int B, hipStream_t s) {
  ProfScope ps(p, PK_RING, B, s);
  const size_t lds = (size_t)4 * p.nlon * sizeof(double2);
  hipLaunchKernelGGL(k_ring_tendency, dim3(p.nlat * B), dim3(kRingThreads), lds, s, p.F, p.G, p.c2,
                     p.w, p.twid, rplan(p), p.M, p.nlon, p.nlat, p.nlat2, B, p.a);
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
    ProfScope ps(p, PK_SRING, nb, s);
    const size_t lds = (size_t)p.nlon * sizeof(double2);
    hipLaunchKernelGGL(k_ring_synth, dim3(p.nlat, (nb + 1) / 2), dim3(kRingThreads), lds, s, p.F,
                       grid + (size_t)b0 * p.nlat * p.nlon, p.twid, rplan(p), p.M, p.nlon, p.nlat,
                       p.nlat2, nb);
    PINT_HIP(hipGetLastError());
  }
  return PINT_OK;
}

pint_status scalar_analysis(Plan& p, const double* grid, double* spec, int B, hipStream_t s) {
  for (int b0 = 0; b0 < B; b0 += p.max_batch) {
    const int nb = (B - b0) < p.max_batch ? (B - b0) : p.max_batch;
    ProfScope ps(p, PK_SRING, nb, s);
    const size_t lds = (size_t)p.nlon * sizeof(double2);
    hipLaunchKernelGGL(k_ring_anal, dim3(p.nlat, (nb + 1) / 2), dim3(kRingThreads), lds, s,
                       grid + (size_t)b0 * p.nlat * p.nlon, p.G, p.w, p.twid, rplan(p), p.M,
                       p.nlon, p.nlat, nb);
    PINT_HIP(hipGetLastError());
    pint_status st = legendre_anal(p, nb, 1, s);
    if (st != PINT_OK) return st;
    st = scalar_post(p, spec + (size_t)b0 * p.ncoef * 2, nb, s);
    if (st != PINT_OK) return st;
  }
  return PINT_OK;
}

}  // namespace pint
