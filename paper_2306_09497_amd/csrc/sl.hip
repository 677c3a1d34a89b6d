// Semi-Lagrangian semi-implicit SETTLS steps (Sec. 2.3.2, eqs.
// SETTLS_trajectories and SL_SI_SETTLS; one-step variant of Sec. 3.2.4).
//
// One step of B states:
//   spectral prep + Legendre synthesis GEMM  (shared with the IMEX path) of
//     U^n and U^{n-1} together (2B states; B in the one-step variant)
//   k_ring_sl_grid   Fourier -> grid: delta, Phi', G, dPhi'/dlambda, U, V
//   k_sl_fields      per grid point: the extrapolated wind 2V^n - V^{n-1},
//                    R_Phi and the wind right-hand side R_V (Cartesian)
//   k_sl_points      per arrival point: SETTLS departure point, bicubic
//                    interpolation of R_Phi and R_V there, the turn of R_V
//                    into the arrival frame, + dt/2 N_R^n
//   k_ring_sl_anal   grid -> Fourier of (R_Phi*, -v*/cos, u*/cos)
//   Legendre analysis GEMM, then (I - dt/2 L) U^{n+1} = rhs per zonal
//     wavenumber with the Crank-Nicolson factors of the IMEX path
//     (k_sp_sl_solve), viscosity fused.
// Grid arrays are [state][field][nlat][nlon] FP64, latitudes north to south.
#include <cmath>

#include <vector>

#include "pint_internal.h"

namespace pint {

constexpr int kSlThreads = 256;

struct SlGeom {
  const double* mu;     // [nlat] sin(lat)
  const double* c2;     // [nlat] cos^2(lat)
  const double* latx;   // [nlat + 4] latitudes with two mirrored rows beyond each pole
  int nlat, nlon;
  double a, omega, phibar, hdt;   // hdt = dt / 2
};

// Longitude sine/cosine of grid column k.
__device__ inline void lon_sc(int k, int nlon, double* s, double* c) {
  sincospi(2.0 * k / nlon, s, c);
}

// Tensor-product cubic Lagrange stencil at (lam, th): rows (with the row
// mirrored across a pole read at longitude + pi) and weights.
struct Stencil {
  int off[4][4];      // offsets into a [nlat][nlon] plane
  double w[4][4];
};

// Cubic Lagrange weights of nodes n at x: one division per weight.
__device__ inline void lagrange4(const double (&n)[4], double x, double (&w)[4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    double num = 1.0, den = 1.0;
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (k != i) {
        num *= x - n[k];
        den *= n[i] - n[k];
      }
    w[i] = num / den;
  }
}

// The same for the nodes -1, 0, 1, 2 (denominators -6, 2, -2, 6).
__device__ inline void lagrange4_unit(double t, double (&w)[4]) {
  const double a = t + 1.0, b = t - 1.0, c = t - 2.0;
  w[0] = t * b * c * (-1.0 / 6.0);
  w[1] = a * b * c * 0.5;
  w[2] = a * t * c * (-0.5);
  w[3] = a * t * b * (1.0 / 6.0);
}

__device__ inline void make_stencil(const SlGeom& g, const double (&x)[3], Stencil& st) {
  const double kTwoPi = 6.283185307179586476925286766559;
  const double kPi = 3.14159265358979323846264338328;
  double lam = atan2(x[1], x[0]);
  if (lam < 0.0) lam += kTwoPi;
  const double th = atan2(x[2], sqrt(x[0] * x[0] + x[1] * x[1]));
  // longitude: nodes -1, 0, 1, 2 around column i
  double xl = lam / (kTwoPi / g.nlon);
  if (xl >= g.nlon) xl -= g.nlon;
  if (!(xl >= 0.0)) xl = 0.0;                      // NaN input: any in-range column
  const int i = (int)floor(xl);
  const double t = xl - i;
  double wk[4];
  lagrange4_unit(t, wk);
  // latitude: interval e of latx (descending) with latx[e] > th >= latx[e+1]
  double ths = th;
  if (!(ths >= -kPi && ths <= kPi)) ths = 0.0;
  int e = (int)floor((0.5 * kPi - ths) * (g.nlat / kPi) - 0.5) + 2;
  e = e < 1 ? 1 : (e > g.nlat + 1 ? g.nlat + 1 : e);
  while (e > 1 && ths >= g.latx[e]) --e;
  while (e < g.nlat + 1 && ths < g.latx[e + 1]) ++e;
  const double nl[4] = {g.latx[e - 1], g.latx[e], g.latx[e + 1], g.latx[e + 2]};
  double wl[4];
  lagrange4(nl, th, wl);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int er = e - 1 + r;
    int row, shift = g.nlon / 2;
    if (er < 2) {
      row = 1 - er;
    } else if (er < g.nlat + 2) {
      row = er - 2;
      shift = 0;
    } else {
      row = 2 * g.nlat + 1 - er;                   // nlat+2 -> nlat-1, nlat+3 -> nlat-2
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      int col = (i - 1 + c + shift) % g.nlon;
      if (col < 0) col += g.nlon;
      st.off[r][c] = row * g.nlon + col;
      st.w[r][c] = wl[r] * wk[c];
    }
  }
}

__device__ inline double interp(const double* __restrict__ f, const Stencil& st) {
  double acc = 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc = acc + st.w[r][c] * f[st.off[r][c]];
  return acc;
}

// Grid-point right-hand sides at t_n.  The synthesised states are two halves
// of B states: U^n of state b is in half `cur`, U^{n-1} in the other half
// when `two`, else U^n itself:
//   f7[0..2] = 2 V^n - V^{n-1}   (Cartesian, m/s)
//   f7[3]    = R_Phi = Phi' - dt/2 Phibar delta + dt/2 (2 N_R^n - N_R^{n-1})
//   f7[4..6] = R_V = V - dt/2 (grad Phi' + f k x V)   (Cartesian)
__global__ __launch_bounds__(kSlThreads) void k_sl_fields(const double* __restrict__ g6,
                                                          double* __restrict__ f7, SlGeom g,
                                                          int B, int two, int cur) {
  const int npts = g.nlat * g.nlon;
  const int pt = blockIdx.x * kSlThreads + threadIdx.x;
  if (pt >= npts) return;
  const int b = blockIdx.y;
  const int j = pt / g.nlon, k = pt - j * g.nlon;
  const int bn = cur * B + b;
  const double* gn = g6 + (size_t)bn * 6 * npts + pt;
  const double* gp = g6 + (size_t)(two ? (1 - cur) * B + b : bn) * 6 * npts + pt;
  const double de = gn[0], ph = gn[npts], G = gn[2 * npts], Pl = gn[3 * npts];
  const double ic = 1.0 / sqrt(g.c2[j]), cs = sqrt(g.c2[j]), sn = g.mu[j];
  const double u = gn[4 * npts] * ic, v = gn[5 * npts] * ic;
  const double up = gp[4 * npts] * ic, vp = gp[5 * npts] * ic;
  const double nr = -ph * de, nrp = -gp[npts] * gp[0];
  const double gl = Pl * ic / g.a, gt = G * ic / g.a;
  const double f = 2.0 * g.omega * sn;
  const double rphi = ph + g.hdt * (-g.phibar * de) + g.hdt * (2.0 * nr - nrp);
  const double ru = u + g.hdt * (-gl + f * v);
  const double rv = v + g.hdt * (-gt - f * u);
  double sl, cl;
  lon_sc(k, g.nlon, &sl, &cl);
  const double ea[3] = {-sl, cl, 0.0};
  const double no[3] = {-sn * cl, -sn * sl, cs};
  double* o = f7 + (size_t)b * 7 * npts + pt;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const double vn = u * ea[d] + v * no[d];
    o[d * npts] = 2.0 * vn - (up * ea[d] + vp * no[d]);
    o[(4 + d) * npts] = ru * ea[d] + rv * no[d];
  }
  o[3 * npts] = rphi;
}

// Departure points and interpolated right-hand sides of every arrival point:
//   o3[0] = R_Phi* + dt/2 N_R^n,  o3[1] = -v* / cos(lat),  o3[2] = u* / cos(lat)
// with (u*, v*) the interpolated R_V turned by the rotation taking the
// departure point to the arrival point, in the arrival's east/north frame.
__global__ __launch_bounds__(kSlThreads) void k_sl_points(const double* __restrict__ g6,
                                                          const double* __restrict__ f7,
                                                          double* __restrict__ o3, SlGeom g,
                                                          int iters, int B, int cur) {
  const int npts = g.nlat * g.nlon;
  // one-dimensional grid of (state, point block) remapped so that every XCD
  // works through one contiguous range: the 16-point gathers of neighbouring
  // arrival points then hit the same L2
  const int nblk = (npts + kSlThreads - 1) / kSlThreads;
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int b = lb / nblk;
  const int pt = (lb - b * nblk) * kSlThreads + threadIdx.x;
  if (pt >= npts) return;
  const int j = pt / g.nlon, k = pt - j * g.nlon;
  const double cs = sqrt(g.c2[j]), sn = g.mu[j], ic = 1.0 / cs;
  double sl, cl;
  lon_sc(k, g.nlon, &sl, &cl);
  const double xa[3] = {cs * cl, cs * sl, sn};
  const double ea[3] = {-sl, cl, 0.0};
  const double no[3] = {-sn * cl, -sn * sl, cs};
  const double* gn = g6 + (size_t)(cur * B + b) * 6 * npts;
  const double u = gn[4 * npts + pt] * ic, v = gn[5 * npts + pt] * ic;
  double vn[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) vn[d] = u * ea[d] + v * no[d];
  const double* F = f7 + (size_t)b * 7 * npts;
  const double h = g.hdt / g.a;
  double xd[3] = {xa[0], xa[1], xa[2]};
  Stencil st;
  for (int it = 0; it < iters; ++it) {
    make_stencil(g, xd, st);
    double y[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) y[d] = xa[d] - h * (interp(F + d * npts, st) + vn[d]);
    const double inv = 1.0 / sqrt(y[0] * y[0] + y[1] * y[1] + y[2] * y[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) xd[d] = y[d] * inv;
  }
  make_stencil(g, xd, st);
  const double rphi = interp(F + 3 * npts, st);
  double r[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) r[d] = interp(F + (4 + d) * npts, st);
  // rotation taking xd to xa: r + w x r + (w (w.r) - |w|^2 r) / (1 + c)
  const double w[3] = {xd[1] * xa[2] - xd[2] * xa[1], xd[2] * xa[0] - xd[0] * xa[2],
                       xd[0] * xa[1] - xd[1] * xa[0]};
  const double c = xd[0] * xa[0] + xd[1] * xa[1] + xd[2] * xa[2];
  const double wr = w[0] * r[0] + w[1] * r[1] + w[2] * r[2];
  const double ww = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
  const double wxr[3] = {w[1] * r[2] - w[2] * r[1], w[2] * r[0] - w[0] * r[2],
                         w[0] * r[1] - w[1] * r[0]};
  double R[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) R[d] = r[d] + wxr[d] + (w[d] * wr - ww * r[d]) / (1.0 + c);
  const double us = R[0] * ea[0] + R[1] * ea[1] + R[2] * ea[2];
  const double vs = R[0] * no[0] + R[1] * no[1] + R[2] * no[2];
  const double nr = -gn[npts + pt] * gn[pt];
  double* o = o3 + (size_t)b * 3 * npts + pt;
  o[0] = rphi + g.hdt * nr;
  o[npts] = -vs * ic;
  o[2 * npts] = us * ic;
}

pint_status sl_check(const Plan& p, const pint_sl_stepper& st, int B, int nsteps) {
  if (p.prec != PINT_FP64) {
    set_error("semi-Lagrangian steps need a PINT_FP64 plan");
    return PINT_E_INVAL;
  }
  if (p.max_batch < 2) {
    set_error("semi-Lagrangian steps need max_batch >= 2");
    return PINT_E_INVAL;
  }
  if (!(st.dt > 0.0) || !std::isfinite(st.dt)) {
    set_error("sl stepper: dt must be positive and finite");
    return PINT_E_INVAL;
  }
  if (st.traj_iters < 0 || st.traj_iters > 64) {
    set_error("sl stepper: traj_iters must be in [0, 64]");
    return PINT_E_INVAL;
  }
  if (st.visc_order < 2 || (st.visc_order & 1) || st.visc_order > 16) {
    set_error("sl stepper: visc_order must be even in [2, 16]");
    return PINT_E_INVAL;
  }
  if (!(st.visc_nu >= 0.0) || !std::isfinite(st.visc_nu)) {
    set_error("sl stepper: visc_nu must be >= 0 and finite");
    return PINT_E_INVAL;
  }
  if (B < 0 || nsteps < 0) {
    set_error("batch and step count must be >= 0");
    return PINT_E_INVAL;
  }
  return PINT_OK;
}

// Scratch of pint_sl_steps on plan p: grid fields of max_batch / 2 state
// pairs, the seven interpolated fields and three results per point, and the
// (I - dt/2 L) factors (a Crank-Nicolson factor set at step 2 dt).
void sl_footprint(const Plan& p, const pint_sl_stepper& st, Footprint& fp) {
  const size_t nbmax = (size_t)(p.max_batch / 2);
  const size_t npts = (size_t)p.nlat * p.nlon;
  fp.need(kSlotSlGrid, 2 * nbmax * 6 * npts);
  fp.need(kSlotSlF, nbmax * 7 * npts);
  fp.need(kSlotSlO, nbmax * 3 * npts);
  fp.factors(fp.cn, 2.0 * st.dt, PINT_T_ALL);
}

pint_status sl_steps(Plan& p, const pint_sl_stepper& st, const double* u_prev, const double* u,
                     double* out, double* out_prev, int B, int nsteps, hipStream_t s) {
  PINT_TRY(sl_check(p, st, B, nsteps));
  if (B == 0) return PINT_OK;
  if (!u || !out || (out_prev && out_prev == out)) {
    set_error("null state array, or out_prev aliasing out");
    return PINT_E_INVAL;
  }
  const size_t sd = (size_t)3 * p.ncoef * 2;   // doubles per state
  const size_t sb = sd * sizeof(double);
  if (nsteps == 0) {
    if (out_prev)
      PINT_HIP(hipMemcpyAsync(out_prev, u_prev ? u_prev : u, B * sb, hipMemcpyDeviceToDevice, s));
    if (out != u) PINT_HIP(hipMemcpyAsync(out, u, B * sb, hipMemcpyDeviceToDevice, s));
    return PINT_OK;
  }
  const int nbmax = p.max_batch / 2;
  const size_t npts = (size_t)p.nlat * p.nlon;
  Footprint fp;
  sl_footprint(p, st, fp);
  DevBuf grid(p, kSlotSlGrid), f7(p, kSlotSlF), o3(p, kSlotSlO);
  PINT_TRY(grid.alloc(fp.slot[kSlotSlGrid]));
  PINT_TRY(f7.alloc(fp.slot[kSlotSlF]));
  PINT_TRY(o3.alloc(fp.slot[kSlotSlO]));
  const CnFactors* f = nullptr;
  PINT_TRY(cn_factors(p, 2.0 * st.dt, PINT_T_ALL, s, &f));   // (I - dt/2 L)
  SlGeom g{p.mu, p.c2, p.sl_lat, p.nlat, p.nlon, p.a, p.omega, p.phibar, 0.5 * st.dt};
  for (int b0 = 0; b0 < B; b0 += nbmax) {
    const int nb = (B - b0) < nbmax ? (B - b0) : nbmax;
    // two halves of nb states: U^n in half `cur`, U^{n-1} in the other; a
    // step writes U^{n+1} over U^{n-1} and flips `cur` (no copies)
    double* half[2] = {p.Ua, p.Ua + (size_t)nb * sd};
    int cur = 0;
    PINT_HIP(hipMemcpyAsync(half[0], u + b0 * sd, nb * sb, hipMemcpyDeviceToDevice, s));
    bool two = u_prev != nullptr;
    if (two)
      PINT_HIP(hipMemcpyAsync(half[1], u_prev + b0 * sd, nb * sb, hipMemcpyDeviceToDevice, s));
    for (int step = 0; step < nsteps; ++step) {
      const bool last = step == nsteps - 1;
      const int nt = two ? 2 * nb : nb;
      PINT_TRY(sp_prep(p, p.Ua, nt, s));
      PINT_TRY(legendre_synth(p, nt, kSynFields, PINT_FP64, s));
      PINT_TRY(ring_sl_grid(p, grid.p, nt, s));
      {
        ProfScope ps(p, PK_SL, nb, s);
        const dim3 lg((unsigned)((npts + kSlThreads - 1) / kSlThreads), (unsigned)nb);
        hipLaunchKernelGGL(k_sl_fields, lg, dim3(kSlThreads), 0, s, grid.p, f7.p, g, nb,
                           two ? 1 : 0, cur);
        hipLaunchKernelGGL(k_sl_points, dim3(lg.x * lg.y), dim3(kSlThreads), 0, s, grid.p, f7.p,
                           o3.p, g, st.traj_iters, nb, cur);
        PINT_HIP(hipGetLastError());
      }
      PINT_TRY(ring_sl_anal(p, o3.p, nb, s));
      PINT_TRY(legendre_anal(p, nb, kAnaFields, PINT_FP64, s));
      double* dst = last ? out + b0 * sd : half[1 - cur];
      PINT_TRY(sp_sl_solve(p, *f, st.dt, st.visc_order, st.visc_nu, dst, nb, s));
      if (last) {
        if (out_prev)
          PINT_HIP(hipMemcpyAsync(out_prev + b0 * sd, half[cur], nb * sb,
                                  hipMemcpyDeviceToDevice, s));
      } else {
        cur = 1 - cur;
        two = true;
      }
    }
  }
  return PINT_OK;
}

}  // namespace pint
