// Spectral-space kernels: layout conversion, synthesis-input preparation,
// tendency assembly with the RK2 stage combine, the Crank-Nicolson solve with
// fused viscosity, the Parareal/MGRIT correction and the increment norms.
// All are HBM-bound streaming kernels over the batch-innermost work layout.
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
// public [B][3][ncoef] <-> work [ncoef][B][3]; one thread per complex element
// ---------------------------------------------------------------------------
__global__ void k_to_work(const double* __restrict__ pub, double* __restrict__ work, int ncoef,
                          int B) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)ncoef * B * 3;
  if (t >= total) return;
  const int f = (int)(t % 3);
  const size_t r = t / 3;
  const int b = (int)(r % B);
  const size_t i = r / B;
  st2(work, t, ld2(pub, ((size_t)b * 3 + f) * ncoef + i));
}

__global__ void k_from_work(const double* __restrict__ work, double* __restrict__ pub, int ncoef,
                            int B) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  const size_t total = (size_t)ncoef * B * 3;
  if (t >= total) return;
  const int i = (int)(t % ncoef);
  const size_t r = t / ncoef;
  const int f = (int)(r % 3);
  const int b = (int)(r / 3);
  st2(pub, t, ld2(work, ((size_t)i * B + b) * 3 + f));
}

pint_status to_work(Plan& p, const double* pub, double* work, int B, hipStream_t s) {
  ProfScope ps(p, PK_LAYOUT, B, s);
  const size_t total = (size_t)p.ncoef * B * 3;
  hipLaunchKernelGGL(k_to_work, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, pub, work,
                     p.ncoef, B);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status from_work(Plan& p, const double* work, double* pub, int B, hipStream_t s) {
  ProfScope ps(p, PK_LAYOUT, B, s);
  const size_t total = (size_t)p.ncoef * B * 3;
  hipLaunchKernelGGL(k_from_work, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, work,
                     pub, p.ncoef, B);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

// ---------------------------------------------------------------------------
// Synthesis inputs (one thread per (row, b)): the coefficients, on Pbar_n^m
// for n = m..M+1, of
//   xi, delta, Phi' (Phi minus the constant Phibar), G = (1-mu^2) dPhi'/dmu,
//   U = u cos(lat) = (1/a)[d chi/d lambda - (1-mu^2) d psi/d mu],
//   V = v cos(lat) = (1/a)[d psi/d lambda + (1-mu^2) d chi/d mu],
// with psi = lap^-1 xi, chi = lap^-1 delta, using
//   (1-mu^2) d/dmu sum_k c_k Pbar_k = sum_n [-(n-1) eps_n c_{n-1} + (n+2) eps_{n+1} c_{n+1}] Pbar_n
// (from (1-mu^2) dPbar_n/dmu = -n eps_{n+1} Pbar_{n+1} + (n+1) eps_n Pbar_{n-1}).
// Output S[row][(b*6 + f)*2 + reim].
// ---------------------------------------------------------------------------
__global__ void k_prep(const double* __restrict__ uw, double* __restrict__ S,
                       const int* __restrict__ rowinfo, int nrows, int M, int B, double a,
                       double phibar) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)nrows * B) return;
  const int b = (int)(t % B);
  const int row = (int)(t / B);
  const int mn = rowinfo[row];
  const int m = mn >> 16, n = mn & 0xffff;
  auto ld = [&](int nn, int f) -> double2 {
    if (nn < m || nn > M) return make_double2(0.0, 0.0);
    return ld2(uw, ((size_t)coef_idx(M, m, nn) * B + b) * 3 + f);
  };
  const double2 ph = ld(n, 0), xi = ld(n, 1), de = ld(n, 2);
  const double2 phm = ld(n - 1, 0), xim = ld(n - 1, 1), dem = ld(n - 1, 2);
  const double2 php = ld(n + 1, 0), xip = ld(n + 1, 1), dep = ld(n + 1, 2);
  const double e0 = eps_nm(n, m), e1 = eps_nm(n + 1, m);
  const double lo = (n - 1) * e0, hi = (n + 2) * e1;
  const double sm = s_of(n - 1, a), s0 = s_of(n, a), sp = s_of(n + 1, a);
  double2 php_ = ph;
  if (m == 0 && n == 0) php_.x -= phibar;
  const double2 G = cadd(cscale(phm, -lo), cscale(php, hi));
  // psi_k = s_k xi_k, chi_k = s_k delta_k
  const double2 psi = cscale(xi, s0), chi = cscale(de, s0);
  const double2 dpsi = cadd(cscale(xim, -lo * sm), cscale(xip, hi * sp));   // (1-mu^2) dpsi/dmu
  const double2 dchi = cadd(cscale(dem, -lo * sm), cscale(dep, hi * sp));
  const double ia = 1.0 / a;
  const double2 U = cscale(csub(cimul(chi, (double)m), dpsi), ia);
  const double2 V = cscale(cadd(cimul(psi, (double)m), dchi), ia);
  double2* out = reinterpret_cast<double2*>(S + ((size_t)row * B + b) * 12);
  out[0] = xi;
  out[1] = de;
  out[2] = php_;
  out[3] = G;
  out[4] = U;
  out[5] = V;
}

// ---------------------------------------------------------------------------
// Tendency assembly and RK2 combine (one thread per (idx, b)).  Q holds, per
// row (m, k <= M+1), the weighted projections
//   Q_f(k) = sum_j w_j Pbar_k^m(mu_j) f_m(mu_j)  for f = N_Phi, K, A/c^2, B/c^2
// (A = xi U, B = xi V, c^2 = 1 - mu^2).  Then
//   N_Phi = Q_NPhi / 2,  K = Q_K / 2,
//   div  = 1/(2a) [ i m Q_A(n) - (-n eps_{n+1} Q_B(n+1) + (n+1) eps_n Q_B(n-1)) ]
//   curl = 1/(2a) [ i m Q_B(n) + (-n eps_{n+1} Q_A(n+1) + (n+1) eps_n Q_A(n-1)) ]
//   N_xi = -div,  N_delta = curl + n(n+1)/a^2 K,   (0,0) of N_xi, N_delta = 0.
// stage 0: out = N; 1: n1 = N, out = ua + dt N; 2: out = ua + dt/2 (n1 + N).
// ---------------------------------------------------------------------------
__global__ void k_assemble(const double* __restrict__ Q, const int* __restrict__ coefmn,
                           const int* __restrict__ rowoff, int ncoef, int M, int B, double a,
                           double dt, int stage, const double* __restrict__ ua,
                           double* __restrict__ n1, double* __restrict__ out) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)ncoef * B) return;
  const int b = (int)(t % B);
  const size_t i = t / B;
  const int mn = coefmn[i];
  const int m = mn >> 16, n = mn & 0xffff;
  auto qrow = [&](int k) -> const double2* {
    const int par = (k - m) & 1;
    const int row = rowoff[2 * m + par] + ((k - m - par) >> 1);
    return reinterpret_cast<const double2*>(Q + ((size_t)row * B + b) * 8);
  };
  const double2* q0 = qrow(n);
  const double2* qp = qrow(n + 1);
  const double2 zero = make_double2(0.0, 0.0);
  double2 qAm = zero, qBm = zero;
  if (n > m) {
    const double2* qm = qrow(n - 1);
    qAm = qm[2];
    qBm = qm[3];
  }
  const double e0 = eps_nm(n, m), e1 = eps_nm(n + 1, m);
  const double ha = 0.5 / a;
  const double2 nphi = cscale(q0[0], 0.5);
  const double2 K = cscale(q0[1], 0.5);
  const double2 hB = cadd(cscale(qp[3], -n * e1), cscale(qBm, (n + 1) * e0));
  const double2 hA = cadd(cscale(qp[2], -n * e1), cscale(qAm, (n + 1) * e0));
  const double2 div = cscale(csub(cimul(q0[2], (double)m), hB), ha);
  const double2 curl = cscale(cadd(cimul(q0[3], (double)m), hA), ha);
  double2 nxi = cscale(div, -1.0);
  double2 nde = cadd(curl, cscale(K, (double)n * (n + 1) / (a * a)));
  if (m == 0 && n == 0) {
    nxi = zero;
    nde = zero;
  }
  const size_t base = (i * B + b) * 3;
  const double2 nv[3] = {nphi, nxi, nde};
  if (stage == 0) {
    for (int f = 0; f < 3; ++f) st2(out, base + f, nv[f]);
  } else if (stage == 1) {
    for (int f = 0; f < 3; ++f) {
      st2(n1, base + f, nv[f]);
      st2(out, base + f, cadd(ld2(ua, base + f), cscale(nv[f], dt)));
    }
  } else {
    const double hdt = 0.5 * dt;
    for (int f = 0; f < 3; ++f)
      st2(out, base + f, cadd(ld2(ua, base + f), cscale(cadd(ld2(n1, base + f), nv[f]), hdt)));
  }
}

pint_status nl_eval(Plan& p, const double* u, double* out, const double* ua, double* n1,
                    double dt, int stage, int B, hipStream_t s) {
  {
    ProfScope ps(p, PK_PREP, B, s);
    const size_t total = (size_t)p.nrows * B;
    hipLaunchKernelGGL(k_prep, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, u, p.S,
                       p.rowinfo, p.nrows, p.M, B, p.a, p.phibar);
    PINT_HIP(hipGetLastError());
  }
  pint_status st = legendre_synth(p, B, kSynFields, s);
  if (st != PINT_OK) return st;
  st = ring_tendency(p, B, s);
  if (st != PINT_OK) return st;
  st = legendre_anal(p, B, kAnaFields, s);
  if (st != PINT_OK) return st;
  {
    ProfScope ps(p, PK_ASSEMBLE, B, s);
    const size_t total = (size_t)p.ncoef * B;
    hipLaunchKernelGGL(k_assemble, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, p.Q,
                       p.coefmn, p.rowoff, p.ncoef, p.M, B, p.a, dt, stage, ua, n1, out);
    PINT_HIP(hipGetLastError());
  }
  return PINT_OK;
}

// ---------------------------------------------------------------------------
// Crank-Nicolson half step (I - alpha L) x = (I + alpha L) y, alpha = dt/4,
// with the viscosity factor 1/(1 + dt nu (n(n+1)/a^2)^(q/2)) applied to the
// result (see cn_factors for the chain form).  One 64-lane wave per (m, b):
//  1. right-hand side r = (I + alpha L) y with Phi eliminated from the delta
//     rows: (r_Phi, r_xi, r_delta + alpha n(n+1)/a^2 r_Phi);
//  2. per chain, forward elimination y_i = alph_i y_{i-1} + invpiv_i r_i and
//     back substitution x_i = gam_i x_{i+1} + y_i.  Each is a first-order
//     linear recurrence, i.e. a composition of affine maps: lane l composes
//     the maps of its SEG consecutive positions, an inclusive scan over the
//     64 lanes (log steps) gives every lane its incoming value, and each lane
//     then runs its own positions;
//  3. x_Phi = r_Phi - alpha Phibar x_delta, viscosity, store.
// The order of operations depends on M only (never on B), so results are
// batch-invariant.  y and x must not overlap.
// ---------------------------------------------------------------------------
__device__ inline double visc_factor(int n, double a, double vdt, double nu, int q) {
  if (!(nu > 0.0)) return 1.0;
  const double l = (double)n * (n + 1) / (a * a);
  double pw = 1.0;
  for (int k = 0; k < q / 2; ++k) pw *= l;
  return 1.0 / (1.0 + vdt * nu * pw);
}

// chain position i of chain c at wavenumber m holds xi if (i even) == (c == 0)
__device__ inline int chain_slot(int i, int chain) { return (((i & 1) == 0) == (chain == 0)) ? 1 : 2; }

__device__ inline double2 cfma(double2 a, double2 x, double2 b) {   // a x + b
  return cadd(cmul(a, x), b);
}

__device__ inline double2 shfl_up2(double2 v, int d) {
  return make_double2(__shfl_up(v.x, d, 64), __shfl_up(v.y, d, 64));
}
__device__ inline double2 shfl_down2(double2 v, int d) {
  return make_double2(__shfl_down(v.x, d, 64), __shfl_down(v.y, d, 64));
}

// Inclusive scan of affine maps f_l(v) = A_l v + B_l over the 64 lanes:
// kUp: lane l gets f_l o f_{l-1} o ... o f_0; otherwise f_l o ... o f_63.
template <bool kUp>
__device__ inline void affine_scan(double2& A, double2& Bv, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const double2 Ap = kUp ? shfl_up2(A, d) : shfl_down2(A, d);
    const double2 Bp = kUp ? shfl_up2(Bv, d) : shfl_down2(Bv, d);
    if (kUp ? lane >= d : lane + d < 64) {
      Bv = cfma(A, Bp, Bv);
      A = cmul(A, Ap);
    }
  }
}

template <int SEG>
__global__ __launch_bounds__(64) void k_cn_solve(
    const double* __restrict__ y, double* __restrict__ x, const double4* __restrict__ co,
    const double2* __restrict__ alph, const double2* __restrict__ gam,
    const double2* __restrict__ invpiv, int M, int ncoef, int B, double a, double W, double lgf,
    double pb, double alpha, double vdt, double nu, int q) {
  const int lb = xcd_remap(blockIdx.x, gridDim.x);    // logical block m * B + b
  const int m = lb / B, b = lb - m * B;
  const int K = M - m + 1;
  const int i0 = coef_idx(M, m, m);
  const int lane = threadIdx.x;
  const int p0 = lane * SEG;
  auto Y = [&](int i, int f) { return ld2(y, ((size_t)(i0 + i) * B + b) * 3 + f); };
  const double2 zero = make_double2(0.0, 0.0), one = make_double2(1.0, 0.0);
  // 1. right-hand side of the lane's positions
  double2 rphi[SEG], rv[2][SEG];
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int i = p0 + k;
    rphi[k] = zero;
    rv[0][k] = zero;
    rv[1][k] = zero;
    if (i < K) {
      const double4 c = co[i0 + i];
      const double A = W * c.x, Bc = W * c.y, C = W * c.z, lap = lgf * c.w;
      const double2 yphi = Y(i, 0), yxi = Y(i, 1), yde = Y(i, 2);
      double2 axi = cimul(yxi, Bc), ade = cadd(cscale(yphi, lap), cimul(yde, Bc));
      if (i > 0) {
        axi = cadd(axi, cscale(Y(i - 1, 2), A));
        ade = csub(ade, cscale(Y(i - 1, 1), A));
      }
      if (i + 1 < K) {
        axi = cadd(axi, cscale(Y(i + 1, 2), C));
        ade = csub(ade, cscale(Y(i + 1, 1), C));
      }
      const double2 rxi = cadd(yxi, cscale(axi, alpha));
      const double2 rde = cadd(yde, cscale(ade, alpha));
      rphi[k] = csub(yphi, cscale(yde, alpha * pb));
      const double2 rdp = cadd(rde, cscale(rphi[k], alpha * lap));
      const bool xi0 = chain_slot(i, 0) == 1;
      rv[0][k] = xi0 ? rxi : rdp;
      rv[1][k] = xi0 ? rdp : rxi;
    }
  }
  // 2. the two chains
#pragma unroll
  for (int ch = 0; ch < 2; ++ch) {
    const size_t fb = (size_t)ch * ncoef + i0;
    double2 al[SEG], be[SEG], ga[SEG];
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      const int i = p0 + k;
      al[k] = i < K ? alph[fb + i] : one;
      ga[k] = i < K ? gam[fb + i] : one;
      be[k] = i < K ? cmul(invpiv[fb + i], rv[ch][k]) : zero;
    }
    // forward: the lane's composite map, scan, then its own positions
    double2 A = one, Bv = zero;
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      Bv = cfma(al[k], Bv, be[k]);
      A = cmul(al[k], A);
    }
    affine_scan<true>(A, Bv, lane);
    double2 v = shfl_up2(Bv, 1);
    if (lane == 0) v = zero;
#pragma unroll
    for (int k = 0; k < SEG; ++k) {
      v = cfma(al[k], v, be[k]);
      rv[ch][k] = p0 + k < K ? v : zero;               // y_i
    }
    // backward (positions beyond K keep the identity map and y = 0)
    A = one;
    Bv = zero;
#pragma unroll
    for (int k = SEG - 1; k >= 0; --k) {
      Bv = cfma(ga[k], Bv, rv[ch][k]);
      A = cmul(ga[k], A);
    }
    affine_scan<false>(A, Bv, lane);
    v = shfl_down2(Bv, 1);
    if (lane == 63) v = zero;
#pragma unroll
    for (int k = SEG - 1; k >= 0; --k) {
      v = cfma(ga[k], v, rv[ch][k]);
      rv[ch][k] = v;                                   // x_i
    }
  }
  // 3. Phi, viscosity, store
#pragma unroll
  for (int k = 0; k < SEG; ++k) {
    const int i = p0 + k;
    if (i < K) {
      const bool xi0 = chain_slot(i, 0) == 1;
      const double2 xxi = xi0 ? rv[0][k] : rv[1][k];
      const double2 xde = xi0 ? rv[1][k] : rv[0][k];
      const double vf = visc_factor(m + i, a, vdt, nu, q);
      const double2 xphi = csub(rphi[k], cscale(xde, alpha * pb));
      const size_t g = ((size_t)(i0 + i) * B + b) * 3;
      st2(x, g, cscale(xphi, vf));
      st2(x, g + 1, cscale(xxi, vf));
      st2(x, g + 2, cscale(xde, vf));
    }
  }
}

pint_status cn_apply(Plan& p, const CnFactors& f, double dt, unsigned terms, int q, double nu,
                     const double* y, double* x, int B, hipStream_t s) {
  ProfScope ps(p, PK_CN, B, s);
  const double W = (terms & PINT_T_LC) ? 2.0 * p.omega : 0.0;
  const bool lg = (terms & PINT_T_LG) != 0;
  const double pb = lg ? p.phibar : 0.0;
  const double nuv = (terms & PINT_T_VISC) ? nu : 0.0;
  const double alpha = dt / 4.0;
  const int K = p.M + 1;
  const dim3 grid((unsigned)(K * B));
#define PINT_CN(SEG)                                                                            \
  hipLaunchKernelGGL(k_cn_solve<SEG>, grid, dim3(64), 0, s, y, x, p.cnco, f.alph, f.gam,       \
                     f.invpiv, p.M, p.ncoef, B, p.a, W, lg ? 1.0 : 0.0, pb, alpha, dt, nuv, q)
  if (K <= 64) {
    PINT_CN(1);
  } else if (K <= 128) {
    PINT_CN(2);
  } else if (K <= 256) {
    PINT_CN(4);
  } else if (K <= 512) {
    PINT_CN(8);
  } else {
    set_error("Crank-Nicolson chains longer than 512 are not supported (M=%d)", p.M);
    return PINT_E_INVAL;
  }
#undef PINT_CN
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

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

}  // namespace pint
