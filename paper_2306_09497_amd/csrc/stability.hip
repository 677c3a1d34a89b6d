// Stability maps of Sec. 4 on the device: max |A| over a grid of xi_N for
// the scalar test equation u' = (lambda_L + lambda_N) u, for a time stepper
// alone or for two-level MGRIT with F(CF)^nu relaxation (nu = 0: Parareal)
// with an IMEX fine propagator and an IMEX or SL-SI-SETTLS coarse one.
//
//   IMEX (Sec. 4.1.1, Heun keeping U*):
//       A = ((4 + xi_L)/(4 - xi_L))^2 (1 + xi_N (2 + xi_N)/2)
//   SL-SI-SETTLS (eq. stability_SL_SI_SETTLS): both roots of
//       (1 - xi_L/2) A^2 - (e^{-i ks}(1 + xi_L/2 + xi_N) + xi_N/2) A
//           + (xi_N/2) e^{-i ks} = 0,   ks = 2 pi j / n_ks, j = 0..n_ks
//   MGRIT (recurrence eq. parareal_FCF_nrelax_B solved in closed form):
//       sum_{i=0}^{k} C(n - i nu, i) S^i R^(n - i(nu+1)),
//       S = F^nu (F - R), F = A_IMEX(xi/cf)^(cf N_c), R = A_c^(N_c)
// xi_L and the grid's xi_N are on the coarse step; the fine propagator takes
// cf N_c steps at xi / cf.  One thread per grid point; pure FP64 ALU work.
#include <math.h>
#include <vector>

#include "pint_internal.h"

namespace pint {
namespace {

struct Cx {
  double x, y;
};
__device__ inline Cx mk(double x, double y) { return Cx{x, y}; }
__device__ inline Cx add(Cx a, Cx b) { return mk(a.x + b.x, a.y + b.y); }
__device__ inline Cx sub(Cx a, Cx b) { return mk(a.x - b.x, a.y - b.y); }
__device__ inline Cx mul(Cx a, Cx b) { return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline Cx scl(Cx a, double s) { return mk(a.x * s, a.y * s); }
__device__ inline Cx dvd(Cx a, Cx b) {   // Smith's division
  if (fabs(b.x) >= fabs(b.y)) {
    const double r = b.y / b.x, d = b.x + b.y * r;
    return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  const double r = b.x / b.y, d = b.x * r + b.y;
  return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ inline Cx csqrt(Cx z) {         // principal branch
  const double r = hypot(z.x, z.y);
  if (r == 0.0) return mk(0.0, 0.0);
  const double t = sqrt(0.5 * (r + fabs(z.x)));
  if (z.x >= 0.0) return mk(t, z.y / (2.0 * t));
  return mk(fabs(z.y) / (2.0 * t), copysign(t, z.y));
}
__device__ inline Cx cpow(Cx x, int n) {   // binary exponentiation, n >= 0
  Cx r = mk(1.0, 0.0), p = x;
  for (unsigned m = (unsigned)n; m; m >>= 1) {
    if (m & 1u) r = mul(r, p);
    p = mul(p, p);
  }
  return r;
}
__device__ inline Cx imex_amp(Cx xl, Cx xn) {
  const Cx ai = dvd(add(mk(4.0, 0.0), xl), sub(mk(4.0, 0.0), xl));
  const Cx e = add(mk(1.0, 0.0), scl(mul(xn, add(mk(2.0, 0.0), xn)), 0.5));
  return mul(mul(ai, ai), e);
}

constexpr int kMaxK = 64;

struct StabArgs {
  int kind, coarse, n, k, cf, nc, nu, n_ks, nre, nim;
  double xlr, xli, re0, dre, im0, dim;
  double binom[kMaxK + 1];   // C(n - i nu, i)
};

__device__ double mgrit_abs(const StabArgs& a, Cx F, Cx R) {
  const Cx S = mul(cpow(F, a.nu), sub(F, R));
  Cx s = mk(0.0, 0.0);
  for (int i = 0; i <= a.k; ++i) {
    const int e = a.n - i * (a.nu + 1);
    if (e < 0) break;
    s = add(s, scl(mul(cpow(S, i), cpow(R, e)), a.binom[i]));
  }
  return hypot(s.x, s.y);
}

__global__ void k_stability_map(StabArgs a, double* __restrict__ out) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x, r = blockIdx.y;
  if (c >= a.nre) return;
  const Cx xl = mk(a.xlr, a.xli);
  const Cx xn = mk(a.re0 + c * a.dre, a.im0 + r * a.dim);
  Cx F = mk(0.0, 0.0);
  if (a.kind == 1) {
    const double icf = 1.0 / a.cf;
    F = cpow(imex_amp(scl(xl, icf), scl(xn, icf)), a.cf * a.nc);
  }
  double worst = 0.0;
  if (a.coarse == 0) {
    const Cx A = imex_amp(xl, xn);
    worst = a.kind == 0 ? hypot(A.x, A.y) : mgrit_abs(a, F, cpow(A, a.nc));
  } else {
    const Cx qa = sub(mk(1.0, 0.0), scl(xl, 0.5));
    for (int j = 0; j <= a.n_ks; ++j) {
      double sn, cs;
      sincos(2.0 * M_PI * j / a.n_ks, &sn, &cs);
      const Cx e = mk(cs, -sn);                       // exp(-i ks)
      const Cx qb = scl(add(mul(e, add(add(mk(1.0, 0.0), scl(xl, 0.5)), xn)), scl(xn, 0.5)), -1.0);
      const Cx qc = mul(scl(xn, 0.5), e);
      const Cx d = csqrt(sub(mul(qb, qb), scl(mul(qa, qc), 4.0)));
      const Cx den = scl(qa, 2.0);
      const Cx roots[2] = {dvd(add(scl(qb, -1.0), d), den), dvd(sub(scl(qb, -1.0), d), den)};
      for (int q = 0; q < 2; ++q) {
        const double v = a.kind == 0 ? hypot(roots[q].x, roots[q].y)
                                     : mgrit_abs(a, F, cpow(roots[q], a.nc));
        worst = fmax(worst, v);
      }
    }
  }
  out[(size_t)r * a.nre + c] = worst;
}

}  // namespace
}  // namespace pint

using namespace pint;

extern "C" pint_status pint_stability_map(const pint_stability_cfg* cfg, double* out,
                                          void* stream) {
  if (!cfg || !out) {
    set_error("null config or output");
    return PINT_E_INVAL;
  }
  const pint_stability_cfg& c = *cfg;
  if ((c.kind != 0 && c.kind != 1) || (c.coarse != 0 && c.coarse != 1) || c.nre < 1 ||
      c.nim < 1 || c.nim > 65535 || (double)c.nre * c.nim > (double)(1 << 28) || c.n < 0 || c.k < 0 ||
      c.k > kMaxK || c.cfactor < 1 || c.n_c < 1 || c.nrelax < 0 || c.nrelax > 8 ||
      (c.coarse == 1 && c.n_ks < 1)) {
    set_error("pint_stability_map: need kind 0/1, coarse 0/1, nre >= 1, 1 <= nim <= 65535, nre nim <= 2^28, "
              "n >= 0, 0 <= k <= %d, cfactor, n_c >= 1, 0 <= nrelax <= 8, n_ks >= 1 for "
              "SL-SI-SETTLS", kMaxK);
    return PINT_E_INVAL;
  }
  StabArgs a{};
  a.kind = c.kind;
  a.coarse = c.coarse;
  a.n = c.n;
  a.k = c.k;
  a.cf = c.cfactor;
  a.nc = c.n_c;
  a.nu = c.nrelax;
  a.n_ks = c.n_ks;
  a.nre = c.nre;
  a.nim = c.nim;
  a.xlr = c.xl_re;
  a.xli = c.xl_im;
  a.re0 = c.re0;
  a.im0 = c.im0;
  a.dre = c.nre > 1 ? (c.re1 - c.re0) / (c.nre - 1) : 0.0;
  a.dim = c.nim > 1 ? (c.im1 - c.im0) / (c.nim - 1) : 0.0;
  for (int i = 0; i <= c.k; ++i) {   // C(n - i nu, i), 0 when i > n - i nu
    const int m = c.n - i * c.nrelax;
    double b = m >= i ? 1.0 : 0.0;
    for (int j = 1; j <= i && m >= i; ++j) b = b * (m - i + j) / j;
    a.binom[i] = b;
  }
  hipLaunchKernelGGL(k_stability_map, dim3((c.nre + 255) / 256, c.nim), dim3(256), 0,
                     (hipStream_t)stream, a, out);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}
