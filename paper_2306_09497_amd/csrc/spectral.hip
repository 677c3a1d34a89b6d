// Spectral-space kernels: the Crank-Nicolson solve with fused viscosity, the
// synthesis-input preparation and the tendency assembly with the RK2 stage
// combine, fused per zonal wavenumber; the Parareal/MGRIT correction and the
// increment norms.  HBM-bound over the public layout [B][3][ncoef].
#include "pint_internal.h"

namespace pint {

__device__ inline double2 ld2(const double* p, size_t i) {
  return *reinterpret_cast<const double2*>(p + 2 * i);
}
__device__ inline void st2(double* p, size_t i, double2 v) {
  *reinterpret_cast<double2*>(p + 2 * i) = v;
}
__device__ inline double2 cadd(double2 x, double2 y) { return make_double2(x.x + y.x, x.y + y.y); }
__device__ inline double2 csub(double2 x, double2 y) { return make_double2(x.x - y.x, x.y - y.y); }
__device__ inline double2 cscale(double2 x, double s) { return make_double2(x.x * s, x.y * s); }
__device__ inline double2 cimul(double2 x, double s) {   // i * s * x
  return make_double2(-s * x.y, s * x.x);
}

// ---------------------------------------------------------------------------
// Spectral kernels.  States are in the public layout [B][3][ncoef] complex.
// The chain of zonal wavenumber m (positions i = n - m, K = M - m + 1 of
// them) occupies a segment of ceil(K / SEG) consecutive lanes of a 64-lane
// wave; lane slo + l of the segment owns the SEG positions i = l*SEG ..
// l*SEG+SEG-1 (positions >= K hold zeros).  A wave carries one state and
// several chains on disjoint segments (a task: one long chain and the short
// ones that fill the remaining lanes), so that the lanes of high wavenumbers
// are not left idle.  The neighbours n-1 and n+1 that the recurrence shifts
// and the Crank-Nicolson right-hand side need come from the adjacent lanes by
// shuffles, and the Crank-Nicolson scans run over the segment; reads across a
// segment's ends are masked, which gives exactly the values a wave holding
// the chain alone has there (zeros, and identity maps, whose composition is
// exact).  The order of every floating-point operation depends on M only,
// never on B or on the packing, so results are bitwise batch-invariant.
// ---------------------------------------------------------------------------
__device__ inline double2 cfma(double2 a, double2 x, double2 b) {   // a x + b
  return cadd(cmul(a, x), b);
}
__device__ inline double2 shfl_up2(double2 v, int d) {
  return make_double2(__shfl_up(v.x, d, 64), __shfl_up(v.y, d, 64));
}
__device__ inline double2 shfl_down2(double2 v, int d) {
  return make_double2(__shfl_down(v.x, d, 64), __shfl_down(v.y, d, 64));
}

__device__ inline double visc_factor(int n, double a, double vdt, double nu, int q) {
  if (!(nu > 0.0)) return 1.0;
  const double l = (double)n * (n + 1) / (a * a);
  double pw = 1.0;
  for (int k = 0; k < q / 2; ++k) pw *= l;
  return 1.0 / (1.0 + vdt * nu * pw);
}

// chain position i of chain c holds xi if (i even) == (c == 0), else delta
__device__ inline bool xi_on_chain0(int i) { return (i & 1) == 0; }

// Inclusive scan of affine maps f_l(v) = A_l v + B_l over the lanes
// [slo, shi) of a segment: kUp: lane l gets f_l o f_{l-1} o ... o f_slo;
// otherwise f_l o ... o f_{shi-1}.
template <bool kUp>
__device__ inline void affine_scan(double2& A, double2& Bv, int lane, int slo, int shi) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double2 Ap = kUp ? shfl_up2(A, d) : shfl_down2(A, d);
    const double2 Bp = kUp ? shfl_up2(Bv, d) : shfl_down2(Bv, d);
    if (kUp ? lane - d >= slo : lane + d < shi) {
      Bv = cfma(A, Bp, Bv);
      A = cmul(A, Ap);
    }
  }
}

// Where one lane sits: its chain's wavenumber m, the wave's state b, chain
// length K, first packed index i0 of m, the lane, its first position p0 and
// the chain's lane segment [slo, shi).
struct WaveAt {
  int m, b, K, i0, lane, p0, slo, shi;
};

// Position i of the lane clamped to its chain (K >= 1): every load a lane
// makes is then in bounds and issued unconditionally, beside the others of
// its phase, and the value of a position past the chain's end is replaced by
// what it stands for (zero, or an identity map) afterwards.
__device__ inline int clamp_pos(int i, const WaveAt& w) { return i < w.K ? i : w.K - 1; }

// A workgroup holds kSpecWaves waves: the states b0 .. b0+kSpecWaves-1 of one
// task, whose rows of S and Q are adjacent in memory.  Logical block
// task * nbg + bg, XCD-remapped.  A wave past the last state has nothing to do
// (w.b >= B).  Task record: chain count, kSpecTaskChains wavenumbers, their
// first lanes.
constexpr int kSpecWaves = 4;
constexpr int kSpecTaskChains = 8;
constexpr int kSpecTaskInts = 1 + 2 * kSpecTaskChains;

template <int SEG>
__device__ inline WaveAt wave_at(int M, int B, const int* __restrict__ tasks) {
  WaveAt w;
  const int nbg = (B + kSpecWaves - 1) / kSpecWaves;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int t = lb / nbg;
  w.b = (lb - t * nbg) * kSpecWaves + (int)(threadIdx.x >> 6);
  w.lane = threadIdx.x & 63;
  const int* tk = tasks + (size_t)t * kSpecTaskInts;
  const int* lo = tk + 1 + kSpecTaskChains;
  const int n = tk[0];
  int c = 0;
  for (int q = 1; q < n; ++q) c = w.lane >= lo[q] ? q : c;
  w.m = tk[1 + c];
  w.slo = lo[c];
  w.shi = c + 1 < n ? lo[c + 1] : 64;
  w.K = M - w.m + 1;
  w.i0 = coef_idx(M, w.m, w.m);
  w.p0 = (w.lane - w.slo) * SEG;
  return w;
}

template <int SEG>
__device__ inline void load_state(const double* __restrict__ u, const WaveAt& w, int ncoef,
                                  double2 (&V)[SEG][3]) {
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int i = w.p0 + k, ic = clamp_pos(i, w);
#pragma unroll
    for (int f = 0; f < 3; ++f) {
      const double2 v = ld2(u, ((size_t)w.b * 3 + f) * ncoef + w.i0 + ic);
      V[k][f] = i < w.K ? v : make_double2(0.0, 0.0);
    }
  }
}

template <int SEG>
__device__ inline void store_state(double* __restrict__ u, const WaveAt& w, int ncoef,
                                   const double2 (&V)[SEG][3]) {
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int i = w.p0 + k;
    if (i < w.K) {
#pragma unroll
      for (int f = 0; f < 3; ++f) st2(u, ((size_t)w.b * 3 + f) * ncoef + w.i0 + i, V[k][f]);
    }
  }
}

// Values of the positions just before and after the lane's positions (zero
// beyond the ends of its chain's segment).
template <int SEG>
__device__ inline void edge_neighbours(const double2 (&V)[SEG][3], const WaveAt& w,
                                       double2 (&prev)[3], double2 (&next)[3]) {
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    prev[f] = shfl_up2(V[SEG - 1][f], 1);
    next[f] = shfl_down2(V[0][f], 1);
    if (w.lane == w.slo) prev[f] = make_double2(0.0, 0.0);
    if (w.lane == w.shi - 1) next[f] = make_double2(0.0, 0.0);
  }
}

// Crank-Nicolson half step (eq. IMEX_implicit) on the wave's (m, b):
// (I - alpha L) x = (I + alpha L) y with the factor chains of cn_factors, then
// the viscosity factor 1/(1 + vdt nu (n(n+1)/a^2)^(q/2)) (nu = 0: none).
//  1. r = (I + alpha L) y with Phi eliminated from the delta rows:
//     (r_Phi, r_xi, r_delta + alpha n(n+1)/a^2 r_Phi);
//  2. per chain, forward elimination y_i = alph_i y_{i-1} + invpiv_i r_i and
//     back substitution x_i = gam_i x_{i+1} + y_i: each a composition of
//     affine maps, composed per lane, scanned over the lanes, then finished
//     per lane;
//  3. x_Phi = r_Phi - alpha Phibar x_delta and the viscosity factor.
struct CnArgs {
  const double4* co;
  const double2 *alph, *gam, *invpiv;
  double a, W, lgf, pb, alpha, vdt, nu;
  int q;
  // the right-hand side is given (semi-Lagrangian step): solve
  // (I - alpha L) x = y instead of (I - alpha L) x = (I + alpha L) y
  int rhs_given;
};

template <int SEG>
__device__ inline void cn_lane(double2 (&V)[SEG][3], const WaveAt& w, int ncoef,
                               const CnArgs& c) {
  const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
  double2 prev[3], next[3];
  edge_neighbours<SEG>(V, w, prev, next);
  double2 rphi[SEG], rv[2][SEG];
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int i = w.p0 + k;
    rphi[k] = zero;
    rv[0][k] = zero;
    rv[1][k] = zero;
    const double2 xim = k > 0 ? V[k - 1][1] : prev[1], dem = k > 0 ? V[k - 1][2] : prev[2];
    const double2 xip = k + 1 < SEG ? V[k + 1][1] : next[1];
    const double2 dep = k + 1 < SEG ? V[k + 1][2] : next[2];
    const double4 cf = c.co[w.i0 + clamp_pos(i, w)];
    if (i < w.K) {
      const double A = c.W * cf.x, Bc = c.W * cf.y, C = c.W * cf.z, lap = c.lgf * cf.w;
      const double2 yphi = V[k][0], yxi = V[k][1], yde = V[k][2];
      double2 axi = cimul(yxi, Bc), ade = cadd(cscale(yphi, lap), cimul(yde, Bc));
      if (i > 0) {
        axi = cadd(axi, cscale(dem, A));
        ade = csub(ade, cscale(xim, A));
      }
      if (i + 1 < w.K) {
        axi = cadd(axi, cscale(dep, C));
        ade = csub(ade, cscale(xip, C));
      }
      const double ex = c.rhs_given ? 0.0 : c.alpha;
      const double2 rxi = cadd(yxi, cscale(axi, ex));
      const double2 rde = cadd(yde, cscale(ade, ex));
      rphi[k] = csub(yphi, cscale(yde, ex * c.pb));
      const double2 rdp = cadd(rde, cscale(rphi[k], c.alpha * lap));
      rv[0][k] = xi_on_chain0(i) ? rxi : rdp;
      rv[1][k] = xi_on_chain0(i) ? rdp : rxi;
    }
  }
#pragma unroll
  for (int ch = 0; ch < 2; ++ch) {
    const size_t fb = (size_t)ch * ncoef + w.i0;
    double2 al[SEG], be[SEG], ga[SEG];
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      const int i = w.p0 + k, ic = clamp_pos(i, w);
      const double2 a0 = c.alph[fb + ic], g0 = c.gam[fb + ic], p0 = c.invpiv[fb + ic];
      al[k] = i < w.K ? a0 : one;
      ga[k] = i < w.K ? g0 : one;
      be[k] = i < w.K ? cmul(p0, rv[ch][k]) : zero;
    }
    double2 A = one, Bv = zero;
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      Bv = cfma(al[k], Bv, be[k]);
      A = cmul(al[k], A);
    }
    affine_scan<true>(A, Bv, w.lane, w.slo, w.shi);
    double2 v = shfl_up2(Bv, 1);
    if (w.lane == w.slo) v = zero;
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      v = cfma(al[k], v, be[k]);
      rv[ch][k] = w.p0 + k < w.K ? v : zero;          // y_i
    }
    A = one;
    Bv = zero;
#pragma unroll
    for (int k = SEG - 1; k >= 0; --k) {
      Bv = cfma(ga[k], Bv, rv[ch][k]);
      A = cmul(ga[k], A);
    }
    affine_scan<false>(A, Bv, w.lane, w.slo, w.shi);
    v = shfl_down2(Bv, 1);
    if (w.lane == w.shi - 1) v = zero;
#pragma unroll
    for (int k = SEG - 1; k >= 0; --k) {
      v = cfma(ga[k], v, rv[ch][k]);
      rv[ch][k] = v;                                    // x_i
    }
  }
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int i = w.p0 + k;
    if (i < w.K) {
      const double2 xxi = xi_on_chain0(i) ? rv[0][k] : rv[1][k];
      const double2 xde = xi_on_chain0(i) ? rv[1][k] : rv[0][k];
      const double vf = visc_factor(w.m + i, c.a, c.vdt, c.nu, c.q);
      V[k][0] = cscale(csub(rphi[k], cscale(xde, c.alpha * c.pb)), vf);
      V[k][1] = cscale(xxi, vf);
      V[k][2] = cscale(xde, vf);
    } else {
      V[k][0] = V[k][1] = V[k][2] = zero;
    }
  }
}

// Synthesis inputs (Sec. 2.1-2.2) of the wave's (m, b): the coefficients, on
// Pbar_n^m for n = m..M+1, of
//   xi, delta, Phi' (Phi minus the constant Phibar), G = (1-mu^2) dPhi'/dmu,
//   U = u cos(lat) = (1/a)[d chi/d lambda - (1-mu^2) d psi/d mu],
//   V = v cos(lat) = (1/a)[d psi/d lambda + (1-mu^2) d chi/d mu],
// with psi = lap^-1 xi, chi = lap^-1 delta, using
//   (1-mu^2) d/dmu sum_k c_k Pbar_k = sum_n [-(n-1) eps_n c_{n-1} + (n+2) eps_{n+1} c_{n+1}] Pbar_n
// (from (1-mu^2) dPbar_n/dmu = -n eps_{n+1} Pbar_{n+1} + (n+1) eps_n Pbar_{n-1}).
// Row n = M+1 (state zero there) is written by the lane holding n = M.
// Output S[row][(b*6 + f)*2 + reim], stored in the Legendre GEMM's element
// type SE (FP64, or FP32 in the mixed-precision mode).
__device__ inline void put_c(double* p, double2 v) { *reinterpret_cast<double2*>(p) = v; }
__device__ inline void put_c(float* p, double2 v) {
  *reinterpret_cast<float2*>(p) = make_float2((float)v.x, (float)v.y);
}
__device__ inline double2 get_c(const double* p) { return *reinterpret_cast<const double2*>(p); }
__device__ inline double2 get_c(const float* p) {
  const float2 f = *reinterpret_cast<const float2*>(p);
  return make_double2((double)f.x, (double)f.y);
}

template <typename SE>
__device__ inline void prep_row(SE* __restrict__ S, const int* __restrict__ rowoff, int m,
                                int n, int b, int B, double a, double phibar, const double2* cur,
                                const double2* pv, const double2* nx) {
  const double2 xi = cur[1], de = cur[2];
  double2 ph = cur[0];
  if (m == 0 && n == 0) ph.x -= phibar;
  const double e0 = eps_nm(n, m), e1 = eps_nm(n + 1, m);
  const double lo = (n - 1) * e0, hi = (n + 2) * e1;
  const double sm = s_of(n - 1, a), s0 = s_of(n, a), sp = s_of(n + 1, a);
  const double2 G = cadd(cscale(pv[0], -lo), cscale(nx[0], hi));
  const double2 psi = cscale(xi, s0), chi = cscale(de, s0);
  const double2 dpsi = cadd(cscale(pv[1], -lo * sm), cscale(nx[1], hi * sp));
  const double2 dchi = cadd(cscale(pv[2], -lo * sm), cscale(nx[2], hi * sp));
  const double ia = 1.0 / a;
  const double2 U = cscale(csub(cimul(chi, (double)m), dpsi), ia);
  const double2 V = cscale(cadd(cimul(psi, (double)m), dchi), ia);
  const int par = (n - m) & 1;
  const int row = rowoff[2 * m + par] + ((n - m - par) >> 1);
  SE* out = S + ((size_t)row * B + b) * 12;
  put_c(out + 0, xi);
  put_c(out + 2, de);
  put_c(out + 4, ph);
  put_c(out + 6, G);
  put_c(out + 8, U);
  put_c(out + 10, V);
}

template <int SEG, typename SE>
__device__ inline void prep_lane(const double2 (&V)[SEG][3], const WaveAt& w, int B,
                                 SE* __restrict__ S, const int* __restrict__ rowoff,
                                 double a, double phibar) {
  double2 prev[3], next[3];
  edge_neighbours<SEG>(V, w, prev, next);
  const double2 zero3[3] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0),
                            make_double2(0.0, 0.0)};
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int i = w.p0 + k;
    if (i < w.K) {
      const double2* pv = k > 0 ? V[k - 1] : prev;
      const double2* nx = k + 1 < SEG ? V[k + 1] : next;
      prep_row(S, rowoff, w.m, w.m + i, w.b, B, a, phibar, V[k], pv, nx);
      if (i + 1 == w.K) prep_row(S, rowoff, w.m, w.m + w.K, w.b, B, a, phibar, zero3, V[k], zero3);
    }
  }
}

// Tendencies from the analysis output Q (Sec. 2.1-2.2).  Q holds, per row
// (m, k <= M+1), the weighted projections
//   Q_f(k) = sum_j w_j Pbar_k^m(mu_j) f_m(mu_j)  for f = N_Phi, K, A/c^2, B/c^2
// (A = xi U, B = xi V, c^2 = 1 - mu^2).  Then
//   N_Phi = Q_NPhi / 2,  K = Q_K / 2,
//   div  = 1/(2a) [ i m Q_A(n) - (-n eps_{n+1} Q_B(n+1) + (n+1) eps_n Q_B(n-1)) ]
//   curl = 1/(2a) [ i m Q_B(n) + (-n eps_{n+1} Q_A(n+1) + (n+1) eps_n Q_A(n-1)) ]
//   N_xi = -div,  N_delta = curl + n(n+1)/a^2 K,   (0,0) of N_xi, N_delta = 0.
template <int SEG, typename SE>
__device__ inline void asm_lane(const SE* __restrict__ Q, const int* __restrict__ rowoff,
                                const WaveAt& w, int B, double a, double2 (&N)[SEG][3]) {
  const double2 zero = make_double2(0.0, 0.0);
  const int m = w.m;
  auto qrow = [&](int k) -> const SE* {
    const int par = (k - m) & 1;
    const int row = rowoff[2 * m + par] + ((k - m - par) >> 1);
    return Q + ((size_t)row * B + w.b) * 8;
  };
  // each row once: (N_Phi, K, A, B) of the lane's positions; A and B of the
  // neighbouring positions n - 1, n + 1 come from the lane itself or from
  // the adjacent lanes of the chain's segment, and the row after the chain's
  // last position (n = M + 1) is read by every lane (one address per chain)
  // and used by the lane that holds that position
  double2 q[SEG][4];
  const SE* rn = qrow(m + w.K);
  const double2 extA = get_c(rn + 4), extB = get_c(rn + 6);
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int i = w.p0 + k;
    const SE* r = qrow(m + clamp_pos(i, w));
#pragma unroll
    for (int f = 0; f < 4; ++f) {
      const double2 v = get_c(r + 2 * f);
      q[k][f] = i < w.K ? v : zero;
    }
  }
  double2 pvA = shfl_up2(q[SEG - 1][2], 1), pvB = shfl_up2(q[SEG - 1][3], 1);
  double2 nxA = shfl_down2(q[0][2], 1), nxB = shfl_down2(q[0][3], 1);
  if (w.lane == w.slo) pvA = pvB = zero;
  if (w.lane == w.shi - 1) nxA = nxB = zero;
  const double ha = 0.5 / a;
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int i = w.p0 + k, n = m + i;
    N[k][0] = N[k][1] = N[k][2] = zero;
    if (i < w.K) {
      const double2 qAm = k > 0 ? q[k - 1][2] : pvA;        // zero at n = m
      const double2 qBm = k > 0 ? q[k - 1][3] : pvB;
      double2 qAp = k + 1 < SEG ? q[k + 1][2] : nxA;
      double2 qBp = k + 1 < SEG ? q[k + 1][3] : nxB;
      if (i + 1 == w.K) {
        qAp = extA;
        qBp = extB;
      }
      const double e0 = eps_nm(n, m), e1 = eps_nm(n + 1, m);
      const double2 Kc = cscale(q[k][1], 0.5);
      const double2 hB = cadd(cscale(qBp, -n * e1), cscale(qBm, (n + 1) * e0));
      const double2 hA = cadd(cscale(qAp, -n * e1), cscale(qAm, (n + 1) * e0));
      const double2 div = cscale(csub(cimul(q[k][2], (double)m), hB), ha);
      const double2 curl = cscale(cadd(cimul(q[k][3], (double)m), hA), ha);
      N[k][0] = cscale(q[k][0], 0.5);
      if (!(m == 0 && n == 0)) {
        N[k][1] = cscale(div, -1.0);
        N[k][2] = cadd(curl, cscale(Kc, (double)n * (n + 1) / (a * a)));
      }
    }
  }
}

struct SpecArgs {
  const int* rowoff;
  const int* tasks;
  int M, ncoef, B;
  double a, phibar;
};

// K_A: Ua = CN(in); S = synthesis input of Ua.
template <int SEG, typename SE>
__global__ __launch_bounds__(64 * kSpecWaves) void k_sp_cn_prep(const double* __restrict__ in,
                                                   double* __restrict__ ua, SE* __restrict__ S,
                                                   SpecArgs sa, CnArgs c) {
  const WaveAt w = wave_at<SEG>(sa.M, sa.B, sa.tasks);
  if (w.b >= sa.B) return;                            // uniform per wave
  double2 V[SEG][3];
  load_state<SEG>(in, w, sa.ncoef, V);
  cn_lane<SEG>(V, w, sa.ncoef, c);
  store_state<SEG>(ua, w, sa.ncoef, V);
  prep_lane<SEG>(V, w, sa.B, S, sa.rowoff, sa.a, sa.phibar);
}

// K_B (first explicit stage): N1 = N(Q); S = synthesis input of Ua + dt N1.
template <int SEG, typename SE>
__global__ __launch_bounds__(64 * kSpecWaves) void k_sp_stage1(const SE* __restrict__ Q,
                                                  const double* __restrict__ ua,
                                                  double* __restrict__ n1, SE* __restrict__ S,
                                                  double dt, SpecArgs sa) {
  const WaveAt w = wave_at<SEG>(sa.M, sa.B, sa.tasks);
  if (w.b >= sa.B) return;                            // uniform per wave
  double2 N[SEG][3], V[SEG][3];
  asm_lane<SEG>(Q, sa.rowoff, w, sa.B, sa.a, N);
  store_state<SEG>(n1, w, sa.ncoef, N);
  load_state<SEG>(ua, w, sa.ncoef, V);
#pragma unroll
  for (int k = 0; k < SEG; ++k)
#pragma unroll
    for (int f = 0; f < 3; ++f) V[k][f] = cadd(V[k][f], cscale(N[k][f], dt));
  prep_lane<SEG>(V, w, sa.B, S, sa.rowoff, sa.a, sa.phibar);
}

// K_C (second explicit stage and the closing half step):
// U = D_nu CN(Ua + dt/2 (N1 + N(Q))); chain = 0: out = U; chain = 1: the next
// step's first half step follows at once: ua = CN(U), S = its synthesis input.
// With a correction (corr != null) the step is the coarse propagation of a
// PinT sweep: out holds G_old on entry and receives U, and
// corr = (U - G_old) + f, the update pr_update makes (bitwise); chain then
// starts the next sweep step from corr.
template <int SEG, typename SE>
__global__ __launch_bounds__(64 * kSpecWaves) void k_sp_stage2(const SE* __restrict__ Q,
                                                  double* __restrict__ ua,
                                                  const double* __restrict__ n1,
                                                  double* __restrict__ out,
                                                  SE* __restrict__ S, double dt, int chain,
                                                  const double* __restrict__ cf,
                                                  double* __restrict__ corr,
                                                  SpecArgs sa, CnArgs c) {
  const WaveAt w = wave_at<SEG>(sa.M, sa.B, sa.tasks);
  if (w.b >= sa.B) return;                            // uniform per wave
  double2 N[SEG][3], V[SEG][3];
  asm_lane<SEG>(Q, sa.rowoff, w, sa.B, sa.a, N);
  load_state<SEG>(n1, w, sa.ncoef, V);
  const double hdt = 0.5 * dt;
#pragma unroll
  for (int k = 0; k < SEG; ++k)
#pragma unroll
    for (int f = 0; f < 3; ++f) N[k][f] = cadd(V[k][f], N[k][f]);   // N1 + N
  load_state<SEG>(ua, w, sa.ncoef, V);
#pragma unroll
  for (int k = 0; k < SEG; ++k)
#pragma unroll
    for (int f = 0; f < 3; ++f) V[k][f] = cadd(V[k][f], cscale(N[k][f], hdt));
  cn_lane<SEG>(V, w, sa.ncoef, c);                    // with the stepper's viscosity
  if (corr) {
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      const int i = w.p0 + k;
      if (i < w.K) {
#pragma unroll
        for (int f = 0; f < 3; ++f) {
          const size_t at = ((size_t)w.b * 3 + f) * sa.ncoef + w.i0 + i;
          const double2 go = ld2(out, at), fv = ld2(cf, at);
          const double2 cv = cadd(csub(V[k][f], go), fv);
          st2(corr, at, cv);
          st2(out, at, V[k][f]);
          V[k][f] = cv;                 // a chained step continues from corr
        }
      }
    }
  }
  if (chain) {
    CnArgs c1 = c;
    c1.nu = 0.0;
    cn_lane<SEG>(V, w, sa.ncoef, c1);
    store_state<SEG>(ua, w, sa.ncoef, V);
    prep_lane<SEG>(V, w, sa.B, S, sa.rowoff, sa.a, sa.phibar);
  } else if (!corr) {
    store_state<SEG>(out, w, sa.ncoef, V);
  }
}

// Synthesis input of the states in (pint_tendency).
template <int SEG, typename SE>
__global__ __launch_bounds__(64 * kSpecWaves) void k_sp_prep(const double* __restrict__ in,
                                                SE* __restrict__ S, SpecArgs sa) {
  const WaveAt w = wave_at<SEG>(sa.M, sa.B, sa.tasks);
  if (w.b >= sa.B) return;                            // uniform per wave
  double2 V[SEG][3];
  load_state<SEG>(in, w, sa.ncoef, V);
  prep_lane<SEG>(V, w, sa.B, S, sa.rowoff, sa.a, sa.phibar);
}

// N(Q) to out (pint_tendency).
template <int SEG, typename SE>
__global__ __launch_bounds__(64 * kSpecWaves) void k_sp_tend(const SE* __restrict__ Q,
                                                double* __restrict__ out, SpecArgs sa) {
  const WaveAt w = wave_at<SEG>(sa.M, sa.B, sa.tasks);
  if (w.b >= sa.B) return;                            // uniform per wave
  double2 N[SEG][3];
  asm_lane<SEG>(Q, sa.rowoff, w, sa.B, sa.a, N);
  store_state<SEG>(out, w, sa.ncoef, N);
}

// out = CN(in) (c0), then, if two, out = CN(out) (c1): pint_implicit and the
// linear-only IMEX step.
template <int SEG>
__global__ __launch_bounds__(64 * kSpecWaves) void k_sp_cn(const double* __restrict__ in,
                                              double* __restrict__ out, int two, SpecArgs sa,
                                              CnArgs c0, CnArgs c1) {
  const WaveAt w = wave_at<SEG>(sa.M, sa.B, sa.tasks);
  if (w.b >= sa.B) return;                            // uniform per wave
  double2 V[SEG][3];
  load_state<SEG>(in, w, sa.ncoef, V);
  cn_lane<SEG>(V, w, sa.ncoef, c0);
  if (two) cn_lane<SEG>(V, w, sa.ncoef, c1);
  store_state<SEG>(out, w, sa.ncoef, V);
}

// Semi-Lagrangian step (Sec. 2.3.2, eq. SL_SI_SETTLS): the analysed
// departure-point right-hand side (R_Phi*, curl R_V*, div R_V*) -> U^{n+1}
// solving (I - dt/2 L) U^{n+1} = rhs, then the viscosity.  Q holds the
// analysis of (R_Phi*, K = 0, A, B) with (A, B) = (-v*, u*) / cos(lat), so
// that the assembly's (-div, curl) of (A, B) is (curl, div) of (u*, v*).
template <int SEG>
__global__ __launch_bounds__(64 * kSpecWaves) void k_sp_sl_solve(const double* __restrict__ Q,
                                                    double* __restrict__ out, SpecArgs sa,
                                                    CnArgs c) {
  const WaveAt w = wave_at<SEG>(sa.M, sa.B, sa.tasks);
  if (w.b >= sa.B) return;                            // uniform per wave
  double2 V[SEG][3];
  asm_lane<SEG, double>(Q, sa.rowoff, w, sa.B, sa.a, V);
  if (w.m == 0 && w.lane == w.slo) V[0][0].x += sa.phibar;   // Phi = Phibar + Phi'
  cn_lane<SEG>(V, w, sa.ncoef, c);
  store_state<SEG>(out, w, sa.ncoef, V);
}

// ---- launchers ----
static int seg_of(int M) {
  const int K = M + 1;
  return K <= 64 ? 1 : K <= 128 ? 2 : K <= 256 ? 4 : K <= 512 ? 8 : 0;
}

// A single state (the serial sweep) runs one wave per workgroup: the other
// three waves of a four-state workgroup would have nothing to do.
static unsigned spec_threads(int B) { return B == 1 ? 64u : 64u * kSpecWaves; }

// Workgroups of a launch over B states: tasks x state groups.
static unsigned spec_grid(const Plan& p, int B) {
  return (unsigned)(p.n_spec_tasks * ((B + kSpecWaves - 1) / kSpecWaves));
}

// Tasks: the chains in order of decreasing length, each opening a task that
// the shortest chains not yet placed then fill while their segments fit in
// the 64 lanes (at most kSpecTaskChains chains per task).  A function of M
// (and the lanes per chain) only.
pint_status spec_tasks_build(Plan& p, size_t* total) {
  const int seg = seg_of(p.M) > 0 ? seg_of(p.M) : 64;   // unsupported M: launches refuse
  auto lanes = [&](int m) { return (p.M - m + 1 + seg - 1) / seg; };
  std::vector<int> h;
  for (int i = 0, j = p.M; i <= j;) {
    int rec[kSpecTaskInts] = {};
    int n = 0, used = 0;
    auto add = [&](int m) {
      rec[1 + n] = m;
      rec[1 + kSpecTaskChains + n] = used;
      used += lanes(m);
      ++n;
    };
    add(i++);
    while (j >= i && n < kSpecTaskChains && used + lanes(j) <= 64) add(j--);
    rec[0] = n;
    h.insert(h.end(), rec, rec + kSpecTaskInts);
  }
  p.n_spec_tasks = (int)(h.size() / kSpecTaskInts);
  void* d = nullptr;
  hipError_t e = hipMalloc(&d, h.size() * sizeof(int));
  if (e != hipSuccess) {
    set_error("hipMalloc(%zu bytes) failed: %s", h.size() * sizeof(int), hipGetErrorString(e));
    return PINT_E_NOMEM;
  }
  p.spec_tasks = static_cast<int*>(d);
  if (total) *total += h.size() * sizeof(int);
  PINT_HIP(hipMemcpy(d, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
  return PINT_OK;
}

static SpecArgs spec_args(const Plan& p, int B) {
  SpecArgs sa;
  sa.rowoff = p.rowoff;
  sa.tasks = p.spec_tasks;
  sa.M = p.M;
  sa.ncoef = p.ncoef;
  sa.B = B;
  sa.a = p.a;
  sa.phibar = p.phibar;
  return sa;
}

static CnArgs cn_args(const Plan& p, const CnFactors& f, const pint_stepper& st, bool visc) {
  CnArgs c;
  c.co = p.cnco;
  c.alph = f.alph;
  c.gam = f.gam;
  c.invpiv = f.invpiv;
  c.a = p.a;
  c.W = (st.terms & PINT_T_LC) ? 2.0 * p.omega : 0.0;
  const bool lg = (st.terms & PINT_T_LG) != 0;
  c.lgf = lg ? 1.0 : 0.0;
  c.pb = lg ? p.phibar : 0.0;
  c.alpha = st.dt / 4.0;
  c.vdt = st.dt;
  c.nu = (visc && (st.terms & PINT_T_VISC)) ? st.visc_nu : 0.0;
  c.q = st.visc_order;
  c.rhs_given = 0;
  return c;
}

// launch(SEG, SE): SEG coefficients per lane, SE the element type of the
// Legendre GEMM operands S and Q (FP32 in the mixed-precision modes).
#define PINT_SEG_DISPATCH(launch)                                                   \
  switch (seg_of(p.M) * (p.prec != PINT_FP64 ? -1 : 1)) {                           \
    case 1: launch(1, double); break;                                               \
    case 2: launch(2, double); break;                                               \
    case 4: launch(4, double); break;                                               \
    case 8: launch(8, double); break;                                               \
    case -1: launch(1, float); break;                                               \
    case -2: launch(2, float); break;                                               \
    case -4: launch(4, float); break;                                               \
    case -8: launch(8, float); break;                                               \
    default:                                                                        \
      set_error("chains longer than 512 coefficients are not supported (M=%d)", p.M); \
      return PINT_E_INVAL;                                                          \
  }

pint_status sp_cn_prep(Plan& p, const CnFactors& f, const pint_stepper& st, const double* in,
                       int B, hipStream_t s) {
  ProfScope ps(p, PK_CN, B, s);
  const SpecArgs sa = spec_args(p, B);
  const CnArgs c = cn_args(p, f, st, false);
  const dim3 grid(spec_grid(p, B));
#define L(SEG, SE)                                                                      \
  hipLaunchKernelGGL((k_sp_cn_prep<SEG, SE>), grid, dim3(spec_threads(B)), 0, s, in, p.Ua, \
                     reinterpret_cast<SE*>(p.S), sa, c)
  PINT_SEG_DISPATCH(L)
#undef L
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status sp_stage1(Plan& p, double dt, int B, hipStream_t s) {
  ProfScope ps(p, PK_ASSEMBLE, B, s);
  const SpecArgs sa = spec_args(p, B);
  const dim3 grid(spec_grid(p, B));
#define L(SEG, SE)                                                                    \
  hipLaunchKernelGGL((k_sp_stage1<SEG, SE>), grid, dim3(spec_threads(B)), 0, s,          \
                     reinterpret_cast<const SE*>(p.Q), p.Ua, p.N1, reinterpret_cast<SE*>(p.S), \
                     dt, sa)
  PINT_SEG_DISPATCH(L)
#undef L
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status sp_stage2(Plan& p, const CnFactors& f, const pint_stepper& st, double* out,
                      bool chain, int B, hipStream_t s, const double* cf, double* corr) {
  ProfScope ps(p, PK_ASSEMBLE, B, s);
  const SpecArgs sa = spec_args(p, B);
  const CnArgs c = cn_args(p, f, st, true);
  const dim3 grid(spec_grid(p, B));
#define L(SEG, SE)                                                                    \
  hipLaunchKernelGGL((k_sp_stage2<SEG, SE>), grid, dim3(spec_threads(B)), 0, s,          \
                     reinterpret_cast<const SE*>(p.Q), p.Ua, p.N1, out,                  \
                     reinterpret_cast<SE*>(p.S), st.dt, chain ? 1 : 0, cf, corr, sa, c)
  PINT_SEG_DISPATCH(L)
#undef L
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status sp_prep(Plan& p, const double* in, int B, hipStream_t s) {
  ProfScope ps(p, PK_PREP, B, s);
  const SpecArgs sa = spec_args(p, B);
  const dim3 grid(spec_grid(p, B));
#define L(SEG, SE)                                                                 \
  hipLaunchKernelGGL((k_sp_prep<SEG, SE>), grid, dim3(spec_threads(B)), 0, s, in,      \
                     reinterpret_cast<SE*>(p.S), sa)
  PINT_SEG_DISPATCH(L)
#undef L
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status sp_tend(Plan& p, double* out, int B, hipStream_t s) {
  ProfScope ps(p, PK_ASSEMBLE, B, s);
  const SpecArgs sa = spec_args(p, B);
  const dim3 grid(spec_grid(p, B));
#define L(SEG, SE)                                                                 \
  hipLaunchKernelGGL((k_sp_tend<SEG, SE>), grid, dim3(spec_threads(B)), 0, s,          \
                     reinterpret_cast<const SE*>(p.Q), out, sa)
  PINT_SEG_DISPATCH(L)
#undef L
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status sp_cn(Plan& p, const CnFactors& f, const pint_stepper& st0, const pint_stepper* st1,
                  const double* in, double* out, int B, hipStream_t s) {
  ProfScope ps(p, PK_CN, B, s);
  const SpecArgs sa = spec_args(p, B);
  const CnArgs c0 = cn_args(p, f, st0, st1 == nullptr);
  const CnArgs c1 = st1 ? cn_args(p, f, *st1, true) : c0;
  const int two = st1 ? 1 : 0;
  const dim3 grid(spec_grid(p, B));
#define L(SEG, SE)                                                                           \
  hipLaunchKernelGGL(k_sp_cn<SEG>, grid, dim3(spec_threads(B)), 0, s, in, out, two, sa, c0, c1)
  PINT_SEG_DISPATCH(L)
#undef L
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}
#undef PINT_SEG_DISPATCH

// ---------------------------------------------------------------------------
// Parareal / MGRIT correction: out = (gnew - gold) + f  (coarse difference
// first, so an unchanged coarse input returns f bitwise).
// ---------------------------------------------------------------------------
__global__ void k_pr_update(const double* __restrict__ gnew, const double* __restrict__ gold,
                            const double* __restrict__ f, double* __restrict__ out, size_t n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  out[t] = (gnew[t] - gold[t]) + f[t];
}

pint_status pr_update(Plan& p, const double* gnew, const double* gold, const double* f,
                      double* out, size_t n, hipStream_t s) {
  ProfScope ps(p, PK_PINT, 1, s);
  hipLaunchKernelGGL(k_pr_update, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, gnew, gold,
                     f, out, n);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

// ---------------------------------------------------------------------------
// Relative differences of state pairs (stopping test and diagnostics): one
// block per state b, fixed-order reduction, sums of w |a - c|^2 and w |a|^2
// for Phi' (m-weight w = 1 for m = 0, 2 otherwise; (0,0) excluded), xi,
// delta, and the wind, whose mean square is sum_{n>=1} w a^2/(n(n+1))
// (|xi|^2 + |delta|^2).  out[b] = {num, den} x {Phi', xi, delta, wind}.
// ---------------------------------------------------------------------------
__global__ void k_rel_diff(const double* __restrict__ a, const double* __restrict__ c,
                           double* __restrict__ out, const int* __restrict__ coefmn, int ncoef,
                           double rad) {
  const int b = blockIdx.x;
  const double* pa = a + (size_t)b * 3 * ncoef * 2;
  const double* pc = c + (size_t)b * 3 * ncoef * 2;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = threadIdx.x; i < ncoef; i += blockDim.x) {
    const int mn = coefmn[i];
    const int m = mn >> 16, n = mn & 0xffff;
    const double w = m == 0 ? 1.0 : 2.0;
    const double kw = n > 0 ? w * rad * rad / ((double)n * (n + 1)) : 0.0;
    for (int f = 0; f < 3; ++f) {
      const size_t o = ((size_t)f * ncoef + i) * 2;
      const double ar = pa[o], ai = pa[o + 1];
      const double dr = ar - pc[o], di = ai - pc[o + 1];
      const double dd = dr * dr + di * di, aa = ar * ar + ai * ai;
      const double wf = (f == 0 && i == 0) ? 0.0 : w;
      acc[2 * f] += wf * dd;
      acc[2 * f + 1] += wf * aa;
      if (f > 0) {
        acc[6] += kw * dd;
        acc[7] += kw * aa;
      }
    }
  }
  __shared__ double sh[8][256];
  for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] = acc[q];
  __syncthreads();
  for (int h = blockDim.x / 2; h > 0; h >>= 1) {
    if (threadIdx.x < h)
      for (int q = 0; q < 8; ++q) sh[q][threadIdx.x] += sh[q][threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x < 8) out[8 * b + threadIdx.x] = sh[threadIdx.x][0];
}

pint_status rel_diff(Plan& p, const double* a, const double* c, double* out_host, int B,
                     hipStream_t s) {
  for (int b0 = 0; b0 < B; b0 += p.max_batch) {
    const int nb = (B - b0) < p.max_batch ? (B - b0) : p.max_batch;
    const size_t off = (size_t)b0 * 3 * p.ncoef * 2;
    ProfScope ps(p, PK_PINT, nb, s);
    hipLaunchKernelGGL(k_rel_diff, dim3(nb), dim3(256), 0, s, a + off, c + off, p.red, p.coefmn,
                       p.ncoef, p.a);
    PINT_HIP(hipGetLastError());
    PINT_HIP(hipMemcpyAsync(p.h_red, p.red, (size_t)nb * 8 * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    PINT_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nb * 4; ++i) {
      const double num = p.h_red[2 * i], den = p.h_red[2 * i + 1];
      out_host[(size_t)b0 * 4 + i] = den > 0.0 ? sqrt(num / den) : sqrt(num);
    }
  }
  return PINT_OK;
}

// The same sums for B state pairs at once into dev[8 B], copied to the
// pinned host array host[8 B]; nothing waits (graph-capturable).
pint_status rel_diff_enqueue(Plan& p, const double* a, const double* c, double* dev,
                             double* host, int B, hipStream_t s) {
  if (B <= 0) return PINT_OK;
  ProfScope ps(p, PK_PINT, B, s);
  hipLaunchKernelGGL(k_rel_diff, dim3(B), dim3(256), 0, s, a, c, dev, p.coefmn, p.ncoef, p.a);
  PINT_HIP(hipGetLastError());
  PINT_HIP(hipMemcpyAsync(host, dev, (size_t)B * 8 * sizeof(double), hipMemcpyDeviceToHost, s));
  return PINT_OK;
}

// out_host[B][4] from the sums of rel_diff_enqueue, once they have arrived.
void rel_diff_finish(const double* host, double* out_host, int B) {
  for (int i = 0; i < B * 4; ++i) {
    const double num = host[2 * i], den = host[2 * i + 1];
    out_host[i] = den > 0.0 ? sqrt(num / den) : sqrt(num);
  }
}

// ---------------------------------------------------------------------------
// Scalar transforms: coefficients in/out of the GEMM operands (nf = 1).
// ---------------------------------------------------------------------------
__global__ void k_scalar_prep(const double* __restrict__ spec, double* __restrict__ S,
                              const int* __restrict__ rowinfo, int nrows, int M, int ncoef,
                              int B) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)nrows * B) return;
  const int b = (int)(t % B);
  const int row = (int)(t / B);
  const int mn = rowinfo[row];
  const int m = mn >> 16, n = mn & 0xffff;
  double2 v = make_double2(0.0, 0.0);
  if (n <= M) v = ld2(spec, (size_t)b * ncoef + coef_idx(M, m, n));
  st2(S, (size_t)row * B + b, v);
}

__global__ void k_scalar_post(const double* __restrict__ Q, double* __restrict__ spec,
                              const int* __restrict__ coefmn, const int* __restrict__ rowoff,
                              int ncoef, int B) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)ncoef * B) return;
  const int i = (int)(t % ncoef);
  const int b = (int)(t / ncoef);
  const int mn = coefmn[i];
  const int m = mn >> 16, n = mn & 0xffff;
  const int par = (n - m) & 1;
  const int row = rowoff[2 * m + par] + ((n - m - par) >> 1);
  st2(spec, t, cscale(ld2(Q, (size_t)row * B + b), 0.5));
}

pint_status scalar_prep(Plan& p, const double* spec, int B, hipStream_t s) {
  const size_t total = (size_t)p.nrows * B;
  hipLaunchKernelGGL(k_scalar_prep, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, spec,
                     p.S, p.rowinfo, p.nrows, p.M, p.ncoef, B);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status scalar_post(Plan& p, double* spec, int B, hipStream_t s) {
  const size_t total = (size_t)p.ncoef * B;
  hipLaunchKernelGGL(k_scalar_post, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, p.Q,
                     spec, p.coefmn, p.rowoff, p.ncoef, B);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

// ---------------------------------------------------------------------------
// Spectral restriction / prolongation between truncations Mf >= Mc (spatial
// coarsening of the coarse levels, Sec. 5): truncate keeps the coefficients
// (m, n) with n <= Mc; pad puts a truncation-Mc state into the
// truncation-Mf packing with zeros above Mc.  One thread per output
// coefficient: x = n - m, y = m, z = state * 3 + field; public layout
// [B][3][ncoef][2].
// ---------------------------------------------------------------------------
__global__ void k_truncate(const double* __restrict__ in, double* __restrict__ out, int Mf,
                           int Mc) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x, m = blockIdx.y, bf = blockIdx.z;
  if (k > Mc - m) return;
  const size_t ncf = (size_t)(Mf + 1) * (Mf + 2) / 2, ncc = (size_t)(Mc + 1) * (Mc + 2) / 2;
  st2(out, bf * ncc + coef_idx(Mc, m, m) + k, ld2(in, bf * ncf + coef_idx(Mf, m, m) + k));
}

__global__ void k_pad(const double* __restrict__ in, double* __restrict__ out, int Mc, int Mf) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x, m = blockIdx.y, bf = blockIdx.z;
  if (k > Mf - m) return;
  const size_t ncf = (size_t)(Mf + 1) * (Mf + 2) / 2, ncc = (size_t)(Mc + 1) * (Mc + 2) / 2;
  const double2 v = (m <= Mc && k <= Mc - m) ? ld2(in, bf * ncc + coef_idx(Mc, m, m) + k)
                                             : make_double2(0.0, 0.0);
  st2(out, bf * ncf + coef_idx(Mf, m, m) + k, v);
}

pint_status spec_truncate(const double* in, int Mf, double* out, int Mc, int B, hipStream_t s) {
  if (B <= 0) return PINT_OK;
  const dim3 grid((unsigned)((Mc + 64) / 64), (unsigned)(Mc + 1), (unsigned)(3 * B));
  hipLaunchKernelGGL(k_truncate, grid, dim3(64), 0, s, in, out, Mf, Mc);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status spec_pad(const double* in, int Mc, double* out, int Mf, int B, hipStream_t s) {
  if (B <= 0) return PINT_OK;
  const dim3 grid((unsigned)((Mf + 64) / 64), (unsigned)(Mf + 1), (unsigned)(3 * B));
  hipLaunchKernelGGL(k_pad, grid, dim3(64), 0, s, in, out, Mc, Mf);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status sp_sl_solve(Plan& p, const CnFactors& f, double dt, int visc_order, double visc_nu,
                        double* out, int B, hipStream_t s) {
  ProfScope ps(p, PK_CN, B, s);
  const SpecArgs sa = spec_args(p, B);
  pint_stepper st{2.0 * dt, visc_order, visc_nu, PINT_T_ALL};
  CnArgs c = cn_args(p, f, st, true);      // alpha = (2 dt) / 4 = dt / 2
  c.vdt = dt;
  c.rhs_given = 1;
  const dim3 grid(spec_grid(p, B));
  switch (seg_of(p.M)) {
#define L(SEG)                                                                              \
  case SEG:                                                                                 \
    hipLaunchKernelGGL((k_sp_sl_solve<SEG>), grid, dim3(spec_threads(B)), 0, s, p.Q, out, sa, \
                       c);                                                                  \
    break;
    L(1) L(2) L(4) L(8)
#undef L
    default:
      set_error("chains longer than 512 coefficients are not supported (M=%d)", p.M);
      return PINT_E_INVAL;
  }
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

}  // namespace pint
