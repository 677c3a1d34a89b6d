// Public C entry points, the batched IMEX propagator and the PinT drivers.
#include <chrono>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pint_internal.h"

namespace pint {

pint_status check_stepper(const Plan& p, const pint_stepper* st) {
  if (!st) {
    set_error("null stepper");
    return PINT_E_INVAL;
  }
  if (!(st->dt > 0.0) || !isfinite(st->dt)) {
    set_error("stepper dt must be positive and finite (got %g)", st->dt);
    return PINT_E_INVAL;
  }
  if ((st->terms & PINT_T_VISC) && st->visc_nu > 0.0 &&
      (st->visc_order < 2 || (st->visc_order & 1) || st->visc_order > 16)) {
    set_error("viscosity order q must be even, 2 <= q <= 16 (got %d)", st->visc_order);
    return PINT_E_INVAL;
  }
  if (!(st->visc_nu >= 0.0) || !isfinite(st->visc_nu)) {
    set_error("viscosity coefficient must be >= 0 and finite");
    return PINT_E_INVAL;
  }
  if (st->terms & ~15u) {
    set_error("unknown bits in terms mask 0x%x", st->terms);
    return PINT_E_INVAL;
  }
  (void)p;
  return PINT_OK;
}

// nsteps IMEX steps (Sec. 2.3.1, eq. IMEX) of B <= max_batch states:
//   Ua = CN(U); Ub = Ua + dt N(Ua); U' = D_nu CN(Ua + dt/2 (N(Ua) + N(Ub)))
// as  sp_cn_prep, [synthesis, ring, analysis, sp_stage1, synthesis, ring,
// analysis, sp_stage2] per step, where each sp_stage2 but the last also runs
// the next step's first half step.  Without the nonlinear term a step is the
// two half steps alone.  out may alias in.
pint_status imex_steps(Plan& p, const pint_stepper& st, const double* in, double* out, int B,
                       int nsteps, hipStream_t s, const double* cf, double* corr, bool prepped,
                       bool chain_out, const CnFactors* given) {
  if ((corr || prepped) && (nsteps < 1 || !(st.terms & PINT_T_NL))) {
    set_error("internal: a fused correction needs a nonlinear step");
    return PINT_E_INVAL;
  }
  if (chain_out && !corr) {
    set_error("internal: chaining a sweep step needs its correction");
    return PINT_E_INVAL;
  }
  if (nsteps == 0) {
    if (in != out)
      PINT_HIP(hipMemcpyAsync(out, in, (size_t)B * 3 * p.ncoef * 2 * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    return PINT_OK;
  }
  const CnFactors* f = given;
  if (!f) PINT_TRY(cn_factors(p, st.dt, st.terms, s, &f));
  if (!(st.terms & PINT_T_NL)) {
    for (int k = 0; k < nsteps; ++k) PINT_TRY(sp_cn(p, *f, st, &st, k ? out : in, out, B, s));
    return PINT_OK;
  }
  if (!prepped) PINT_TRY(sp_cn_prep(p, *f, st, in, B, s));
  for (int k = 0; k < nsteps; ++k) {
    PINT_TRY(legendre_synth(p, B, kSynFields, p.prec, s));
    PINT_TRY(ring_tendency(p, B, s));
    PINT_TRY(legendre_anal(p, B, kAnaFields, p.prec, s));
    PINT_TRY(sp_stage1(p, st.dt, B, s));
    PINT_TRY(legendre_synth(p, B, kSynFields, p.prec, s));
    PINT_TRY(ring_tendency(p, B, s));
    PINT_TRY(legendre_anal(p, B, kAnaFields, p.prec, s));
    const bool last = k + 1 == nsteps;
    PINT_TRY(sp_stage2(p, *f, st, out, !last || chain_out, B, s, last ? cf : nullptr,
                       last ? corr : nullptr));
  }
  return PINT_OK;
}

// Propagate B public-layout states by nsteps, in chunks of max_batch.
static pint_status propagate(Plan& p, const pint_stepper& st, const double* in, double* out,
                             int B, int nsteps, hipStream_t s) {
  const size_t sd = (size_t)3 * p.ncoef * 2;
  for (int b0 = 0; b0 < B; b0 += p.max_batch) {
    const int nb = (B - b0) < p.max_batch ? (B - b0) : p.max_batch;
    PINT_TRY(imex_steps(p, st, in + b0 * sd, out + b0 * sd, nb, nsteps, s));
  }
  return PINT_OK;
}

// ---------------------------------------------------------------------------
// PinT drivers.  States are public layout, one per slice boundary.
// ---------------------------------------------------------------------------
// Device scratch of the drivers: slot `slot` of the plan's pool, kept
// between calls and grown (free, then allocate) only when a call needs more
// than any before it, so repeated solves neither allocate nor synchronise on
// frees.  Calls on one plan are ordered on their stream; a plan is not
// shared between concurrent calls.
static double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// The plan the coarse level runs on: the coarse plan, or none (the fine
// plan) when it has the fine plan's truncation and transform precision --
// such a plan computes bitwise what the fine plan does.
static Plan* coarse_plan_of(const Plan& p, const pint_pint_params* q) {
  if (!q || !q->coarse_plan) return nullptr;
  Plan* c = &q->coarse_plan->p;
  return (c->M == p.M && c->prec == p.prec) ? nullptr : c;
}

pint_status check_params(const Plan& p, const pint_pint_params* q) {
  if (!q) {
    set_error("null params");
    return PINT_E_INVAL;
  }
  PINT_TRY(check_stepper(p, &q->fine));
  if (!q->coarse_sl) PINT_TRY(check_stepper(p, &q->coarse));
  if (q->method != 0 && q->method != 1) {
    set_error("method must be 0 (Parareal) or 1 (MGRIT)");
    return PINT_E_INVAL;
  }
  if (q->n_intervals < 1 || q->fine_steps < 1 || q->coarse_steps < 1 || q->max_iter < 0 ||
      q->max_iter > 128 || q->nrelax < 0 || q->nrelax > 8 || !(q->tol >= 0.0) ||
      (q->resume != 0 && q->resume != 1)) {
    set_error("need n_intervals, fine_steps, coarse_steps >= 1, 0 <= max_iter <= 128, "
              "0 <= nrelax <= 8, tol >= 0, resume in {0, 1}");
    return PINT_E_INVAL;
  }
  if (q->coarse_sl) {
    if (q->method != 1 || q->levels == 3 || q->coarse_steps != 1 || q->coarse_plan) {
      set_error("an SL-SI-SETTLS coarse level needs two-level MGRIT (method 1, levels 2), "
                "coarse_steps = 1 and no coarse_plan");
      return PINT_E_INVAL;
    }
    PINT_TRY(sl_check(p, *q->coarse_sl, 1, 1));
  }
  const double DTf = q->fine.dt * q->fine_steps,
               DTc = (q->coarse_sl ? q->coarse_sl->dt : q->coarse.dt) * q->coarse_steps;
  if (fabs(DTf - DTc) > 1e-9 * DTf) {
    set_error("fine (%g s) and coarse (%g s) propagators must span the same interval", DTf, DTc);
    return PINT_E_INVAL;
  }
  if (q->coarse_plan) {
    const Plan& c = q->coarse_plan->p;
    if (c.M > p.M || c.a != p.a || c.omega != p.omega || c.g != p.g || c.phibar != p.phibar) {
      set_error("coarse_plan needs a truncation <= the plan's (%d > %d?) and the same planet and "
                "Phibar", c.M, p.M);
      return PINT_E_INVAL;
    }
  }
  if (q->levels != 0 && q->levels != 2 && q->levels != 3) {
    set_error("levels must be 2 (or 0) or 3");
    return PINT_E_INVAL;
  }
  if (q->levels == 3) {
    if (q->method != 1) {
      set_error("three levels need method 1 (MGRIT)");
      return PINT_E_INVAL;
    }
    if (q->cfactor1 < 2 || q->n_intervals % q->cfactor1 != 0 || q->coarse2_steps < 1 ||
        q->cycles1 < 1 || q->cycles1 > 8) {
      set_error("three levels need cfactor1 >= 2 dividing n_intervals, coarse2_steps >= 1, "
                "1 <= cycles1 <= 8");
      return PINT_E_INVAL;
    }
    PINT_TRY(check_stepper(p, &q->coarse2));
    const double DT2 = q->coarse2.dt * q->coarse2_steps;
    if (fabs(DT2 - q->cfactor1 * DTc) > 1e-9 * DT2) {
      set_error("level-2 propagator (%g s) must span cfactor1 level-1 intervals (%g s)", DT2,
                q->cfactor1 * DTc);
      return PINT_E_INVAL;
    }
  }
  return PINT_OK;
}

// Strided gather/scatter of states: dst[k] = src[k * stride] (in states).
static pint_status copy_states(double* dst, size_t dstride, const double* src, size_t sstride,
                               int count, size_t sd, hipStream_t s) {
  if (count <= 0) return PINT_OK;
  PINT_HIP(hipMemcpy2DAsync(dst, dstride * sd * sizeof(double), src, sstride * sd * sizeof(double),
                            sd * sizeof(double), count, hipMemcpyDeviceToDevice, s));
  return PINT_OK;
}

// Coarse-level propagation: on the plan itself, or with spatial coarsening
// (Sec. 5) on the coarse plan as pad(step(truncate(u))).  side: the serial
// sweep's stream, with the stepping plan's sweep workspace.
struct CoarseProp {
  Plan& p;
  Plan* pc = nullptr;
  DevBuf cin, cin_side;   // truncation-Mc states
  int cap = 0;            // states cin holds
  explicit CoarseProp(Plan& fine)
      : p(fine), cin(fine, kSlotCin), cin_side(fine, kSlotCinSide) {}
  pint_status init(const pint_pint_params* q, int cap_states) {
    pc = coarse_plan_of(p, q);
    if (!pc) return PINT_OK;
    if (same()) return PINT_OK;
    cap = cap_states;
    const size_t sdc = (size_t)3 * pc->ncoef * 2;
    PINT_TRY(cin.alloc(sdc * cap));
    return cin_side.alloc(sdc);
  }
  Plan& stepping() { return pc ? *pc : p; }
  // the coarse level has the fine truncation (no coarse plan, or one that
  // differs only in its transform precision): no truncation or padding
  bool same() const { return !pc || pc->M == p.M; }
  // One sweep step on the sweep stream: gold (G_old in, G out) and
  // out = (G - G_old) + f, with G = Phi_c(in).  Fused into the last
  // propagation kernel when the coarse level has the fine truncation;
  // otherwise propagation, pr_update and a copy.
  // prepped: the previous step already made this step's first half step
  // (it chained); chain_next: make the next step's.  *chained tells whether
  // this step did.
  bool fusable(const pint_stepper& st, int nsteps) const {
    return same() && nsteps >= 1 && (st.terms & PINT_T_NL);
  }
  pint_status sweep_step(const pint_stepper& st, int nsteps, const double* in, double* gold,
                         const double* f, double* out, double* tmp, hipStream_t s,
                         bool prepped = false, bool chain_next = false, bool* chained = nullptr) {
    const size_t sd = (size_t)3 * p.ncoef * 2;
    if (chained) *chained = false;
    if (fusable(st, nsteps)) {
      SideWork sw(stepping());
      if (chained) *chained = chain_next;
      return imex_steps(stepping(), st, in, gold, 1, nsteps, s, f, out, prepped, chain_next);
    }
    PINT_TRY(run(st, nsteps, in, tmp, 1, s, true));
    PINT_TRY(pr_update(p, tmp, gold, f, out, sd, s));
    PINT_HIP(hipMemcpyAsync(gold, tmp, sd * sizeof(double), hipMemcpyDeviceToDevice, s));
    return PINT_OK;
  }
  pint_status run(const pint_stepper& st, int nsteps, const double* in, double* out, int B,
                  hipStream_t s, bool side) {
    if (same()) {
      Plan& sp = stepping();
      if (side) {
        SideWork sw(sp);
        return propagate(sp, st, in, out, B, nsteps, s);
      }
      return propagate(sp, st, in, out, B, nsteps, s);
    }
    const size_t sdf = (size_t)3 * p.ncoef * 2;
    const int chunk = side ? 1 : cap;
    double* cb = side ? cin_side.p : cin.p;
    for (int b0 = 0; b0 < B; b0 += chunk) {
      const int nb = B - b0 < chunk ? B - b0 : chunk;
      PINT_TRY(spec_truncate(in + b0 * sdf, p.M, cb, pc->M, nb, s));
      if (side) {
        SideWork sw(*pc);
        PINT_TRY(propagate(*pc, st, cb, cb, nb, nsteps, s));
      } else {
        PINT_TRY(propagate(*pc, st, cb, cb, nb, nsteps, s));
      }
      PINT_TRY(spec_pad(cb, pc->M, out + b0 * sdf, p.M, nb, s));
    }
    return PINT_OK;
  }
};

// Three-level MGRIT, level-1 part (Sec. 3.2, multilevel recursion): cycles1
// two-level iterations on levels (1, 2) of the level-1 problem
//   w_0 = U_0,  w_i = psi_i(w_{i-1}) = (Phi_1(w_{i-1}) - G_i) + F_i,
// G_i = Phi_1(v_{i-1}) = Gold[i-1], F_i = Phi_0(u_{mi-1}) = Fv[i-1], starting
// from w = v = U.  Level-1 points are held as W[s][j] = w_{m1 j + s} (rows of
// N2 + 1 entries; row s = 0 uses all, rows s > 0 the first N2), so that the
// points at one s of all level-2 intervals form one contiguous batch.  On
// return U[1..N1] = w.
struct Level1Bufs {
  DevBuf W, Fl, Gl, tmp, F2, G2, gz;
  explicit Level1Bufs(Plan& p)
      : W(p, kSlotW), Fl(p, kSlotFl), Gl(p, kSlotGl), tmp(p, kSlotTmp), F2(p, kSlotF2),
        G2(p, kSlotG2), gz(p, kSlotGz) {}
  pint_status alloc(size_t sd, int m1, int N2) {
    const size_t rows = (size_t)m1 * (N2 + 1);
    PINT_TRY(W.alloc(sd * rows));
    PINT_TRY(Fl.alloc(sd * rows));
    PINT_TRY(Gl.alloc(sd * rows));
    PINT_TRY(tmp.alloc(sd * N2));
    PINT_TRY(F2.alloc(sd * N2));
    PINT_TRY(G2.alloc(sd * N2));
    return gz.alloc(sd);
  }
};

static pint_status level1_cycles(Plan& p, const pint_pint_params* q, Level1Bufs& b,
                                 CoarseProp& cp, double* U, const double* Fv,
                                 const double* Gold, pint_report* r, hipStream_t s) {
  const int N1 = q->n_intervals, m1 = q->cfactor1, N2 = N1 / m1;
  const size_t sd = (size_t)3 * p.ncoef * 2;
  const size_t row = (size_t)(N2 + 1);
  auto at = [&](double* base, int sr, int j) { return base + ((size_t)sr * row + j) * sd; };
  // gather W[s][j] = U[m1 j + s]; F and G of point i = m1 j + s >= 1
  for (int sr = 0; sr < m1; ++sr) {
    PINT_TRY(copy_states(at(b.W.p, sr, 0), 1, U + (size_t)sr * sd, m1, sr == 0 ? N2 + 1 : N2, sd,
                         s));
    const int j0 = sr == 0 ? 1 : 0;
    const size_t src = (size_t)(m1 * j0 + sr - 1) * sd;
    PINT_TRY(copy_states(at(b.Fl.p, sr, j0), 1, Fv + src, m1, N2, sd, s));
    PINT_TRY(copy_states(at(b.Gl.p, sr, j0), 1, Gold + src, m1, N2, sd, s));
  }
  const size_t nb = (size_t)N2 * sd;                  // doubles of one batch
  // out = psi applied to row sin (entries 0..N2-1), forcing of row sr from j0
  auto psi_row = [&](int sin, int sr, int j0, double* out) -> pint_status {
    PINT_TRY(cp.run(q->coarse, q->coarse_steps, at(b.W.p, sin, 0), b.tmp.p, N2, s, false));
    r->coarse_steps += (long long)N2 * q->coarse_steps;
    return pr_update(p, b.tmp.p, at(b.Gl.p, sr, j0), at(b.Fl.p, sr, j0), out, nb, s);
  };
  auto f_relax = [&]() -> pint_status {
    for (int sr = 1; sr < m1; ++sr) PINT_TRY(psi_row(sr - 1, sr, 0, at(b.W.p, sr, 0)));
    return PINT_OK;
  };
  for (int cyc = 0; cyc < q->cycles1; ++cyc) {
    PINT_TRY(f_relax());
    for (int it = 0; it < q->nrelax; ++it) {
      PINT_TRY(psi_row(m1 - 1, 0, 1, at(b.W.p, 0, 1)));   // C-relaxation
      PINT_TRY(f_relax());
    }
    // level 2: F2_j = psi(w_{m1 j - 1}), G2_j = Phi_2(v2_{j-1}), j = 1..N2
    PINT_TRY(psi_row(m1 - 1, 0, 1, b.F2.p));
    PINT_TRY(cp.run(q->coarse2, q->coarse2_steps, at(b.W.p, 0, 0), b.G2.p, N2, s, false));
    r->coarse_steps += (long long)N2 * q->coarse2_steps;
    // serial level-2 solve z_j = (Phi_2(z_{j-1}) - G2_j) + F2_j into W[0][j]
    for (int j = 1; j <= N2; ++j) {
      const double* g2 = b.G2.p + (size_t)(j - 1) * sd;
      const double* gnew = g2;                        // Phi_2(z_0) = Phi_2(v2_0)
      if (j > 1) {
        PINT_TRY(cp.run(q->coarse2, q->coarse2_steps, at(b.W.p, 0, j - 1), b.gz.p, 1, s, false));
        r->coarse_steps += q->coarse2_steps;
        gnew = b.gz.p;
      }
      PINT_TRY(pr_update(p, gnew, g2, b.F2.p + (size_t)(j - 1) * sd, at(b.W.p, 0, j), sd, s));
    }
    PINT_TRY(f_relax());
  }
  // scatter w back to the slice states U[1..N1]
  for (int sr = 0; sr < m1; ++sr) {
    const int j0 = sr == 0 ? 1 : 0;
    PINT_TRY(copy_states(U + (size_t)(m1 * j0 + sr) * sd, m1, at(b.W.p, sr, j0), 1, N2, sd, s));
  }
  return PINT_OK;
}

// Pipelined relaxation (two-level MGRIT with one CF pass, two iterations or
// more): the next iteration's C-relaxation FvR[n] = Phi_0^m(U_n) runs on the
// relax stream, chunk by chunk as soon as the serial sweep has written the
// chunk's slice states, beside the rest of the sweep; in the next iteration
// each chunk of the fine propagation first sets its C-points U_{n+1} =
// FvR[n], waiting only for the relaxation chunks it reads (U_N is not set:
// the sweep overwrites it unread).  Same inputs and kernels as the
// relaxation at the start of the iteration, so the same values.  FvR holds
// two generations (iteration parity), so that making the next one never
// overwrites values the current iteration still reads.  It needs its own
// transform workspace (the chunks of the fine propagation and the sweep use
// the plan's two): relax_cap states in six pool slots.
static bool relax_pipelined(const Plan& p, const pint_pint_params* q) {
  return p.pipeline_relax && q->method == 1 && q->levels != 3 && q->nrelax == 1 &&
         q->max_iter >= 2 && !q->coarse_sl;
}
static int relax_chunk(const Plan& p, int N) { return (N + p.sweep_chunks - 1) / p.sweep_chunks; }
static int relax_cap(const Plan& p, int N) {
  const int cs = relax_chunk(p, N);
  return cs < p.max_batch ? cs : p.max_batch;
}
// doubles of the workspace buffers S, F, G, Q, Ua, N1 for `cap` states (as
// the plan's own at max_batch)
static void relax_work_sizes(const Plan& p, int cap, size_t (&n)[6]) {
  n[0] = (size_t)p.nrows * 12 * cap;
  n[1] = (size_t)(p.M + 1) * fourier_pitch<double>(p.nlat, 12 * cap);
  n[2] = (size_t)(p.M + 1) * fourier_pitch<double>(p.nlat, 8 * cap);
  n[3] = (size_t)p.nrows * 8 * cap;
  n[4] = n[5] = (size_t)p.ncoef * cap * 3 * 2;
}

// Points the plan's transform workspace (and its batch limit) at the
// relaxation workspace while in scope (kernels capture the pointers current
// at their enqueue).
struct RelaxWork {
  Plan& p;
  double *S, *F, *G, *Q, *Ua, *N1;
  int mb;
  RelaxWork(Plan& pl, double* const (&w)[6], int cap) : p(pl) {
    S = p.S, F = p.F, G = p.G, Q = p.Q, Ua = p.Ua, N1 = p.N1, mb = p.max_batch;
    p.S = w[0], p.F = w[1], p.G = w[2], p.Q = w[3], p.Ua = w[4], p.N1 = w[5];
    p.max_batch = cap;
  }
  ~RelaxWork() { p.S = S, p.F = F, p.G = G, p.Q = Q, p.Ua = Ua, p.N1 = N1, p.max_batch = mb; }
};

// Device memory pint_solve(q) needs on plan p (the coarse plan's factor sets
// separately): the driver scratch of its pool slots and the Crank-Nicolson
// factors of its steppers.  Every buffer solve() uses is sized here.
pint_status solve_footprint(const Plan& p, const pint_pint_params* q, Footprint& fp,
                            bool pipelined) {
  if (!q) return PINT_OK;
  PINT_TRY(check_params(p, q));
  const size_t N = (size_t)q->n_intervals;
  const size_t sd = (size_t)3 * p.ncoef * 2;
  fp.need(kSlotGold, sd * N);
  fp.need(kSlotFv, sd * N);
  fp.need(kSlotUprev, sd * (N + 1));
  fp.need(kSlotGtmp, sd);
  fp.need(kSlotIncr, 8 * N);                 // increment sums, one iteration
  fp.host_doubles = 8 * N;
  if (pipelined && relax_pipelined(p, q)) {
    fp.need(kSlotFvR, 2 * sd * N);
    size_t n[6];
    relax_work_sizes(p, relax_cap(p, (int)N), n);
    for (int i = 0; i < 6; ++i) fp.need(kSlotRS + i, n[i]);
  }
  const bool three = q->method == 1 && q->levels == 3;
  if (three) {
    const size_t m1 = (size_t)q->cfactor1, N2 = N / m1, rows = m1 * (N2 + 1);
    fp.need(kSlotW, sd * rows);
    fp.need(kSlotFl, sd * rows);
    fp.need(kSlotGl, sd * rows);
    fp.need(kSlotTmp, sd * N2);
    fp.need(kSlotF2, sd * N2);
    fp.need(kSlotG2, sd * N2);
    fp.need(kSlotGz, sd);
  }
  const Plan* pc = coarse_plan_of(p, q);
  if (pc && pc->M != p.M) {
    const size_t sdc = (size_t)3 * pc->ncoef * 2;
    fp.need(kSlotCin, sdc * N);
    fp.need(kSlotCinSide, sdc);
  }
  fp.factors(fp.cn, q->fine.dt, q->fine.terms);
  if (q->coarse_sl) {
    sl_footprint(p, *q->coarse_sl, fp);
    return PINT_OK;
  }
  auto& cc = pc && pc != &p ? fp.cn_coarse : fp.cn;
  fp.factors(cc, q->coarse.dt, q->coarse.terms);
  if (three) fp.factors(cc, q->coarse2.dt, q->coarse2.terms);
  return PINT_OK;
}

static pint_status solve(Plan& p, const pint_pint_params* q, const double* u0, double* U,
                         pint_report* rep, hipStream_t s) {
  PINT_TRY(check_params(p, q));
  const int N = q->n_intervals;
  const size_t sd = (size_t)3 * p.ncoef * 2;
  const size_t sb = sd * sizeof(double);
  pint_report local;
  pint_report* r = rep ? rep : &local;
  memset(r, 0, sizeof *r);
  // the scratch this problem needs (no allocation when reserved before)
  {
    Footprint fp;
    PINT_TRY(solve_footprint(p, q, fp));
    PINT_TRY(reserve(p, coarse_plan_of(p, q), fp, s));
  }
  DevBuf Gold(p, kSlotGold), Fv(p, kSlotFv), Uprev(p, kSlotUprev), Gtmp(p, kSlotGtmp);
  PINT_TRY(Gold.alloc(sd * N));
  PINT_TRY(Fv.alloc(sd * N));
  PINT_TRY(Uprev.alloc(sd * (N + 1)));
  PINT_TRY(Gtmp.alloc(sd));
  std::vector<double> incr((size_t)N * 4);

  const bool mgrit = q->method == 1;
  const int nrelax = mgrit ? q->nrelax : 0;
  const bool three = mgrit && q->levels == 3;
  const bool pipe = relax_pipelined(p, q);
  DevBuf FvR(p, kSlotFvR);
  double* rwork[6] = {};
  const int rcs = relax_chunk(p, N), rcap = relax_cap(p, N);
  if (pipe) {
    PINT_TRY(FvR.alloc(2 * sd * N));
    size_t n[6];
    relax_work_sizes(p, rcap, n);
    for (int i = 0; i < 6; ++i) {
      DevBuf b(p, kSlotRS + i);
      PINT_TRY(b.alloc(n[i]));
      rwork[i] = b.p;
    }
  }
  bool prerelaxed = false;   // this iteration's relaxation is waiting in FvR
  int kit = 0;               // the iteration being enqueued (FvR generation)
  // work on the relax stream not yet ordered before later work on s: joined
  // into s when the solve returns, whichever way it does
  struct RelaxJoin {
    Plan& p;
    hipStream_t s;
    bool pending = false;
    ~RelaxJoin() {
      if (pending && hipEventRecord(p.relax_join_ev, p.relax_stream) == hipSuccess)
        (void)hipStreamWaitEvent(s, p.relax_join_ev, 0);
    }
  } rjoin{p, s};
  Level1Bufs l1(p);
  if (three) PINT_TRY(l1.alloc(sd, q->cfactor1, N / q->cfactor1));
  CoarseProp coarse(p);
  PINT_TRY(coarse.init(q, N));
  // Crank-Nicolson factors of the propagators, made on s before any work
  // goes to the sweep stream
  const CnFactors* cf = nullptr;
  PINT_TRY(cn_factors(p, q->fine.dt, q->fine.terms, s, &cf));
  const pint_sl_stepper* csl = q->coarse_sl;
  if (csl) PINT_TRY(cn_factors(p, 2.0 * csl->dt, PINT_T_ALL, s, &cf));   // (I - dt/2 L)
  else PINT_TRY(cn_factors(coarse.stepping(), q->coarse.dt, q->coarse.terms, s, &cf));
  if (three) PINT_TRY(cn_factors(coarse.stepping(), q->coarse2.dt, q->coarse2.terms, s, &cf));
  if (q->resume) {
    // continue from the iterate held in U; the coarse values of its slice
    // starts are recomputed (bitwise what the previous sweep produced)
    if (nrelax == 0 && !three && !csl) {   // (the SL iteration makes its own)
      PINT_TRY(coarse.run(q->coarse, q->coarse_steps, U, Gold.p, N, s, false));
      r->coarse_steps += (long long)N * q->coarse_steps;
    }
  } else {
    if (U != u0) PINT_HIP(hipMemcpyAsync(U, u0, sb, hipMemcpyDeviceToDevice, s));
    // iteration 0: serial coarse sweep, G_n = phi_c(U_n), U_{n+1} = G_n
    // (SL: the history of the step from U_n is U_{n-1})
    for (int n = 0; n < N; ++n) {
      if (csl)
        PINT_TRY(sl_steps(p, *csl, n > 0 ? U + (n - 1) * sd : nullptr, U + n * sd,
                          Gold.p + n * sd, nullptr, 1, 1, s));
      else
        PINT_TRY(coarse.run(q->coarse, q->coarse_steps, U + n * sd, Gold.p + n * sd, 1, s,
                            false));
      PINT_HIP(hipMemcpyAsync(U + (n + 1) * sd, Gold.p + n * sd, sb, hipMemcpyDeviceToDevice, s));
      r->coarse_steps += q->coarse_steps;
    }
  }
  // One iteration's device work, enqueued on s (and the sweep stream joined
  // back into s): relaxation and batched fine propagation, the serial
  // correction sweep or level-1 cycles, and the increment sums copied to
  // pinned host memory.  Nothing in it waits or allocates, so it can be
  // captured into a graph; while `capturing`, the phase events are left out
  // (the runtime does not take timed events into a capture), and a replayed
  // iteration is timed as a whole around its graph launch.
  DevBuf Incr(p, kSlotIncr);
  PINT_TRY(Incr.alloc((size_t)8 * N));
  bool capturing = false;
  auto rec = [&](hipEvent_t ev, hipStream_t st) -> pint_status {
    if (!capturing) PINT_HIP(hipEventRecord(ev, st));
    return PINT_OK;
  };
  // speculate: also run the next iteration's relaxation beside the sweep
  auto iteration = [&](int first, hipStream_t s, bool speculate) -> pint_status {
    PINT_TRY(rec(p.ph_ev[0], s));
    PINT_HIP(hipMemcpyAsync(Uprev.p, U, sb * (N + 1), hipMemcpyDeviceToDevice, s));
    const double* src = U;   // C-points the fine propagation starts from
    const size_t gen = (size_t)N * sd;
    double* fvr_use = FvR.p + (size_t)(kit & 1) * gen;         // made beside the last sweep
    double* fvr_make = FvR.p + (size_t)((kit + 1) & 1) * gen;  // for the next iteration
    if (nrelax > 0 && prerelaxed) {
      // the CF pass made beside the previous sweep, set chunk by chunk below
      r->fine_slice_steps += (long long)N * q->fine_steps;
    } else if (nrelax > 0) {
      // F(CF)^nu: each CF pass replaces C-point i+1 by Phi_0^m of C-point i
      for (int it = 0; it < nrelax; ++it) {
        PINT_TRY(propagate(p, q->fine, U, Fv.p, N, q->fine_steps, s));
        PINT_HIP(hipMemcpyAsync(U + sd, Fv.p, sb * N, hipMemcpyDeviceToDevice, s));
        r->fine_slice_steps += (long long)N * q->fine_steps;
      }
    }
    if (csl) {
      // two-level MGRIT with an SL-SI-SETTLS coarse level, on s alone:
      // Gold_i = Phi_1(v_i; v_{i-1}), F_i = Phi_0^m(v_i), then the serial
      // solve U_{i+1} = (Phi_1(U_i; U_{i-1}) - Gold_i) + F_i
      PINT_TRY(sl_steps(p, *csl, nullptr, U, Gold.p, nullptr, 1, 1, s));
      if (N > 1) PINT_TRY(sl_steps(p, *csl, U, U + sd, Gold.p + sd, nullptr, N - 1, 1, s));
      r->coarse_steps += N;
      PINT_TRY(propagate(p, q->fine, U, Fv.p, N, q->fine_steps, s));
      r->fine_slice_steps += (long long)N * q->fine_steps;
      PINT_TRY(rec(p.ph_ev[1], s));
      PINT_TRY(pr_update(p, Gold.p, Gold.p, Fv.p, U + sd, sd, s));
      for (int n = 1; n < N; ++n) {
        PINT_TRY(sl_steps(p, *csl, U + (n - 1) * sd, U + n * sd, Gtmp.p, nullptr, 1, 1, s));
        PINT_TRY(pr_update(p, Gtmp.p, Gold.p + n * sd, Fv.p + n * sd, U + (n + 1) * sd, sd, s));
        r->coarse_steps += 1;
      }
      PINT_TRY(rec(p.ph_ev[2], s));
      return rel_diff_enqueue(p, U + sd, Uprev.p + sd, Incr.p, p.h_incr, N, s);
    }
    if (nrelax > 0) {
      // coarse values of the relaxed C-points, Phi_1(v_i): all of them now
      // for three levels; with two levels chunk by chunk below, so that the
      // sweep can start after the first chunk
      if (three) {
        PINT_TRY(coarse.run(q->coarse, q->coarse_steps, U, Gold.p, N, s, false));
        r->coarse_steps += (long long)N * q->coarse_steps;
      }
    }
    if (three) {
      // three levels: Phi_1(v_i) of the (relaxed) C-points, F_i of every
      // interval, then the level-1 problem by cycles on levels (1, 2)
      if (nrelax == 0) {
        PINT_TRY(coarse.run(q->coarse, q->coarse_steps, U, Gold.p, N, s, false));
        r->coarse_steps += (long long)N * q->coarse_steps;
      }
      PINT_TRY(propagate(p, q->fine, U, Fv.p, N, q->fine_steps, s));
      r->fine_slice_steps += (long long)N * q->fine_steps;
      PINT_TRY(rec(p.ph_ev[1], s));
      PINT_TRY(level1_cycles(p, q, l1, coarse, U, Fv.p, Gold.p, r, s));
      PINT_TRY(rec(p.ph_ev[2], s));
    } else {
      // fine propagation of every active slice (the parallel part), in chunks
      // of cs slices; chunk c's event releases the sweep steps that need it
      const int nact = N - first;
      const int cs = (nact + p.sweep_chunks - 1) / p.sweep_chunks;
      const int nchunk = (nact + cs - 1) / cs;
      for (int c = 0; c < nchunk; ++c) {
        const int n0 = first + c * cs;
        const int nb = cs < N - n0 ? cs : N - n0;
        if (nrelax > 0 && prerelaxed) {
          // C-points U_n = FvR[n-1] of this chunk, once the relaxation chunks
          // (of rcs slices) that make them, and those that still read the
          // U_n they overwrite, are done
          const int lo = n0 > 1 ? n0 : 1, hi = n0 + nb;
          if (hi > lo) {
            for (int rc = (lo - 1) / rcs; rc <= (hi - 1) / rcs; ++rc)
              PINT_HIP(hipStreamWaitEvent(s, p.relax_done_ev[rc], 0));
            PINT_HIP(hipMemcpyAsync(U + (size_t)lo * sd, fvr_use + (size_t)(lo - 1) * sd,
                                    sb * (hi - lo), hipMemcpyDeviceToDevice, s));
          }
        }
        if (nrelax > 0) {
          PINT_TRY(coarse.run(q->coarse, q->coarse_steps, src + n0 * sd, Gold.p + n0 * sd, nb, s,
                              false));
          r->coarse_steps += (long long)nb * q->coarse_steps;
        }
        PINT_TRY(propagate(p, q->fine, src + n0 * sd, Fv.p + n0 * sd, nb, q->fine_steps, s));
        PINT_HIP(hipEventRecord(p.chunk_ev[c], s));
      }
      if (nrelax > 0 && prerelaxed) {
        // the last relaxation chunk (whose last value, U_N, was not used)
        PINT_HIP(hipStreamWaitEvent(s, p.relax_done_ev[(N - 1) / rcs], 0));
        rjoin.pending = false;
      }
      PINT_TRY(rec(p.ph_ev[1], s));
      r->fine_slice_steps += (long long)nact * q->fine_steps;
      // serial correction sweep U_{n+1} = (G(U_n^new) - G(U_n^old)) + F(U_n^old)
      // on the sweep stream and workspace, beside the later chunks.  Step n
      // reads F(U_n^old) (chunk (n-first)/cs) and overwrites U_{n+1}, the start
      // of chunk (n+1-first)/cs when it begins one: it waits for both.
      {
        hipStream_t ss = p.side_stream, rs = p.relax_stream;
        int waited = -1;
        bool prepped = false;   // this step's first half step was made by the previous one
        // relaxation chunk c (slices c rcs .. ) once slice states 0..`done`
        // are final on the sweep stream
        const int nrc = speculate ? (N + rcs - 1) / rcs : 0;
        int next_rc = 0;
        auto relax_ready = [&](int done) -> pint_status {
          for (; next_rc < nrc; ++next_rc) {
            const int a = next_rc * rcs, cnt = rcs < N - a ? rcs : N - a;
            if (a + cnt - 1 > done) break;
            PINT_HIP(hipEventRecord(p.relax_ev[next_rc], ss));
            PINT_HIP(hipStreamWaitEvent(rs, p.relax_ev[next_rc], 0));
            {
              RelaxWork rw(p, rwork, rcap);
              PINT_TRY(propagate(p, q->fine, U + (size_t)a * sd, fvr_make + (size_t)a * sd, cnt,
                                 q->fine_steps, rs));
            }
            PINT_HIP(hipEventRecord(p.relax_done_ev[next_rc], rs));
            rjoin.pending = true;
          }
          return PINT_OK;
        };
        for (int n = first; n < N; ++n) {
          int need = (n + 1 - first) / cs;
          if (need > nchunk - 1) need = nchunk - 1;
          while (waited < need) PINT_HIP(hipStreamWaitEvent(ss, p.chunk_ev[++waited], 0));
          PINT_TRY(relax_ready(n));   // U_0 .. U_n are final
          if (n == first) {   // unchanged input: G_new = G_old
            PINT_TRY(pr_update(p, Gold.p + n * sd, Gold.p + n * sd, Fv.p + n * sd,
                               U + (n + 1) * sd, sd, ss));
          } else {
            bool chained = false;
            PINT_TRY(coarse.sweep_step(q->coarse, q->coarse_steps, U + n * sd, Gold.p + n * sd,
                                       Fv.p + n * sd, U + (n + 1) * sd, Gtmp.p, ss, prepped,
                                       n + 1 < N, &chained));
            prepped = chained;
            r->coarse_steps += q->coarse_steps;
          }
        }
        PINT_TRY(relax_ready(N));
        PINT_TRY(rec(p.ph_ev[2], ss));
        PINT_HIP(hipEventRecord(p.join_ev, ss));
      }
      PINT_HIP(hipStreamWaitEvent(s, p.join_ev, 0));
    }
    return rel_diff_enqueue(p, U + sd, Uprev.p + sd, Incr.p, p.h_incr, N, s);
  };

  // Iterations that repeat the same launches (every slice each time: MGRIT,
  // and Parareal resumed from an iterate) run from a HIP graph captured at
  // the second iteration, on the plan's capture stream, and launched into s.
  struct GraphExec {
    hipGraphExec_t e = nullptr;
    ~GraphExec() {
      if (e) (void)hipGraphExecDestroy(e);
    }
  } graph;
  long long g_fine = 0, g_coarse = 0;   // counters of one replayed iteration
  // (not with the pipelined relaxation: its iterations leave work running
  // on the relax stream, which a graph launch would have to wait for)
  bool graphable = (mgrit || q->resume) && p.use_graphs && !p.prof_on &&
                   !(coarse.pc && coarse.pc->prof_on) && !pipe && !csl;
  pint_status result = PINT_OK;
  for (int k = 0; k < q->max_iter; ++k) {
    const double t0 = now_s();
    // slices before `first` are already exact (Parareal); MGRIT recomputes all
    const int first = (mgrit || q->resume) ? 0 : (k < N ? k : N);
    if (first >= N) break;
    // pipelined relaxation: every iteration but the last makes the next one's
    const bool speculate = pipe && k + 1 < q->max_iter;
    kit = k;
    bool replayed = false;
    if (graph.e) {
      PINT_HIP(hipEventRecord(p.ph_ev[0], s));
      PINT_HIP(hipGraphLaunch(graph.e, s));
      r->fine_slice_steps += g_fine;
      r->coarse_steps += g_coarse;
      ++r->graph_iters;
      replayed = true;
    } else if (graphable && k >= 1) {
      // capture (nothing runs while capturing), instantiate, launch; if the
      // runtime refuses any of it the iteration runs as plain launches and
      // the solve does not try again
      const long long f0 = r->fine_slice_steps, c0 = r->coarse_steps;
      hipStream_t cs = p.capture_stream;
      hipGraph_t g = nullptr;
      const bool dbg = getenv("PINT_GRAPH_DEBUG") != nullptr;
      hipError_t e0 = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
      bool ok = e0 == hipSuccess;
      if (dbg) fprintf(stderr, "[graph] begin capture: %s\n", hipGetErrorString(e0));
      if (ok) {
        capturing = true;
        const pint_status st = iteration(first, cs, speculate);
        capturing = false;
        if (dbg && st != PINT_OK) fprintf(stderr, "[graph] iteration: %s\n", last_error());
        const hipError_t e1 = hipStreamEndCapture(cs, &g);
        if (dbg) fprintf(stderr, "[graph] end capture: %s\n", hipGetErrorString(e1));
        ok = e1 == hipSuccess && st == PINT_OK && g != nullptr;
      }
      if (ok) {
        const hipError_t e2 = hipGraphInstantiate(&graph.e, g, nullptr, nullptr, 0);
        if (dbg) fprintf(stderr, "[graph] instantiate: %s\n", hipGetErrorString(e2));
        ok = e2 == hipSuccess;
      }
      if (g) (void)hipGraphDestroy(g);
      if (ok) {
        g_fine = r->fine_slice_steps - f0;
        g_coarse = r->coarse_steps - c0;
        PINT_HIP(hipEventRecord(p.ph_ev[0], s));
        PINT_HIP(hipGraphLaunch(graph.e, s));
        ++r->graph_iters;
        replayed = true;
      } else {
        (void)hipGetLastError();
        graph.e = nullptr;
        graphable = false;
        r->fine_slice_steps = f0;
        r->coarse_steps = c0;
        PINT_TRY(iteration(first, s, speculate));
      }
    } else {
      PINT_TRY(iteration(first, s, speculate));
    }
    prerelaxed = speculate;
    if (replayed) {   // the graph's two phases as one
      PINT_HIP(hipEventRecord(p.ph_ev[1], s));
      PINT_HIP(hipEventRecord(p.ph_ev[2], s));
    }
    PINT_HIP(hipStreamSynchronize(s));
    rel_diff_finish(p.h_incr, incr.data(), N);
    // stopping measure: Phi' and the wind (entries 0 and 3 of each slice)
    double worst = 0.0;
    bool bad = false;
    double fld[4] = {0.0, 0.0, 0.0, 0.0};
    for (int n = 0; n < N; ++n) {
      for (int f = 0; f < 4; ++f) {
        const double v = incr[(size_t)n * 4 + f];
        if (!isfinite(v)) bad = true;
        else {
          if (v > fld[f]) fld[f] = v;
          if ((f == 0 || f == 3) && v > worst) worst = v;
        }
      }
    }
    r->incr[k] = bad ? NAN : worst;
    for (int f = 0; f < 4; ++f) r->incr_field[k][f] = bad ? NAN : fld[f];
    r->seconds[k] = now_s() - t0;
    {
      // all three events are complete (s was synchronised)
      float ms_f = 0.0f, ms_c = 0.0f;
      if (hipEventElapsedTime(&ms_f, p.ph_ev[0], p.ph_ev[1]) != hipSuccess ||
          hipEventElapsedTime(&ms_c, p.ph_ev[0], p.ph_ev[2]) != hipSuccess) {
        (void)hipGetLastError();
        ms_f = ms_c = -1e3f;         // not measurable: reported as -1 s
      }
      r->fine_seconds[k] = 1e-3 * ms_f;
      r->coarse_seconds[k] = 1e-3 * ms_c;
    }
    r->iters = k + 1;
    if (bad || worst > 1e6) {
      set_error("PinT iteration %d diverged (increment %g)", k, worst);
      return PINT_E_DIVERGED;
    }
    if (q->tol > 0.0 && worst <= q->tol) return PINT_OK;
  }
  if (q->tol > 0.0 && r->iters > 0 && r->incr[r->iters - 1] > q->tol) {
    set_error("tolerance %g not reached in %d iterations (last increment %g)", q->tol, r->iters,
              r->incr[r->iters - 1]);
    result = PINT_E_NOTCONV;
  }
  return result;
}

}  // namespace pint

using namespace pint;

#define API_GUARD(plan)                         \
  if (!(plan)) {                                \
    set_error("null plan");                     \
    return PINT_E_INVAL;                        \
  }

static pint_status check_batch(int B, const void* a, const void* b) {
  if (B < 0) {
    set_error("batch must be >= 0");
    return PINT_E_INVAL;
  }
  if (B > 0 && (!a || !b)) {
    set_error("null array");
    return PINT_E_INVAL;
  }
  return PINT_OK;
}

extern "C" {

pint_status pint_plan_create(const pint_config* cfg, void* stream, pint_plan** out) {
  return create(cfg, (hipStream_t)stream, out);
}

pint_status pint_plan_destroy(pint_plan* plan) {
  API_GUARD(plan);
  destroy(plan);
  return PINT_OK;
}

pint_status pint_plan_info(const pint_plan* plan, pint_info* info) {
  API_GUARD(plan);
  if (!info) {
    set_error("null info");
    return PINT_E_INVAL;
  }
  const Plan& p = plan->p;
  info->M = p.M;
  info->nlon = p.nlon;
  info->nlat = p.nlat;
  info->ncoef = p.ncoef;
  info->max_batch = p.max_batch;
  info->state_doubles = (size_t)3 * p.ncoef * 2;
  info->workspace_bytes = p.ws_bytes;
  info->allocations = p.n_allocs;
  for (int k = 0; k < 2; ++k)
    for (int c = 0; c < 2; ++c) {
      info->gemm_shape[k][c] = p.gemm_variant[k][c];
      info->gemm_us[k][c] = 1e3 * p.gemm_tuned_ms[k][c];
    }
  for (int c = 0; c < 2; ++c) {
    info->ring_threads[c] = (c == 0) == (p.ring_variant[c] == 0) ? 256 : 128;
    info->ring_us[c] = 1e3 * p.ring_tuned_ms[c];
  }
  return PINT_OK;
}

static pint_status workload_footprint(const Plan& p, const pint_pint_params* q,
                                      const pint_sl_stepper* sl, Footprint& fp) {
  PINT_TRY(solve_footprint(p, q, fp));
  if (sl) {
    PINT_TRY(sl_check(p, *sl, 0, 0));
    sl_footprint(p, *sl, fp);
  }
  return PINT_OK;
}

pint_status pint_plan_workspace_bytes(const pint_plan* plan, const pint_pint_params* q,
                                      const pint_sl_stepper* sl, size_t* bytes) {
  API_GUARD(plan);
  if (!bytes) {
    set_error("null output");
    return PINT_E_INVAL;
  }
  Footprint fp;
  PINT_TRY(workload_footprint(plan->p, q, sl, fp));
  *bytes = footprint_bytes(plan->p, coarse_plan_of(plan->p, q), fp);
  return PINT_OK;
}

pint_status pint_plan_reserve(pint_plan* plan, const pint_pint_params* q,
                              const pint_sl_stepper* sl, void* stream) {
  API_GUARD(plan);
  Footprint fp;
  PINT_TRY(workload_footprint(plan->p, q, sl, fp));
  Plan* pc = coarse_plan_of(plan->p, q);
  hipStream_t s = (hipStream_t)stream;
  PINT_TRY(reserve(plan->p, pc, fp, s));
  // launch shapes of the Legendre GEMMs for this workload: single states
  // (the serial sweep) and the batched propagation's launches
  const int big = q ? (q->n_intervals < plan->p.max_batch ? q->n_intervals : plan->p.max_batch)
                    : plan->p.max_batch;
  const int states[2] = {1, big};
  PINT_TRY(tune_legendre(plan->p, states, s));
  PINT_TRY(tune_ring(plan->p, states, s));
  if (pc && pc != &plan->p) {
    const int cbig = big < pc->max_batch ? big : pc->max_batch;
    const int cstates[2] = {1, cbig};
    PINT_TRY(tune_legendre(*pc, cstates, s));
    PINT_TRY(tune_ring(*pc, cstates, s));
  }
  return PINT_OK;
}

pint_status pint_grid_coords(pint_plan* plan, double* mu, double* w, void* stream) {
  API_GUARD(plan);
  if (!mu || !w) {
    set_error("null output");
    return PINT_E_INVAL;
  }
  Plan& p = plan->p;
  hipStream_t s = (hipStream_t)stream;
  PINT_HIP(hipMemcpyAsync(mu, p.mu, p.nlat * sizeof(double), hipMemcpyDeviceToHost, s));
  PINT_HIP(hipMemcpyAsync(w, p.w, p.nlat * sizeof(double), hipMemcpyDeviceToHost, s));
  PINT_HIP(hipStreamSynchronize(s));
  return PINT_OK;
}

pint_status pint_synthesis(pint_plan* plan, const double* spec, double* grid, int B, void* stream) {
  API_GUARD(plan);
  PINT_TRY(check_batch(B, spec, grid));
  if (B == 0) return PINT_OK;
  return scalar_synthesis(plan->p, spec, grid, B, (hipStream_t)stream);
}

pint_status pint_analysis(pint_plan* plan, const double* grid, double* spec, int B, void* stream) {
  API_GUARD(plan);
  PINT_TRY(check_batch(B, spec, grid));
  if (B == 0) return PINT_OK;
  return scalar_analysis(plan->p, grid, spec, B, (hipStream_t)stream);
}

pint_status pint_tendency(pint_plan* plan, const double* u, double* n_out, int B, void* stream) {
  API_GUARD(plan);
  PINT_TRY(check_batch(B, u, n_out));
  Plan& p = plan->p;
  hipStream_t s = (hipStream_t)stream;
  const size_t sd = (size_t)3 * p.ncoef * 2;
  for (int b0 = 0; b0 < B; b0 += p.max_batch) {
    const int nb = (B - b0) < p.max_batch ? (B - b0) : p.max_batch;
    PINT_TRY(sp_prep(p, u + b0 * sd, nb, s));
    PINT_TRY(legendre_synth(p, nb, kSynFields, p.prec, s));
    PINT_TRY(ring_tendency(p, nb, s));
    PINT_TRY(legendre_anal(p, nb, kAnaFields, p.prec, s));
    PINT_TRY(sp_tend(p, n_out + b0 * sd, nb, s));
  }
  return PINT_OK;
}

pint_status pint_implicit(pint_plan* plan, const pint_stepper* st, const double* u, double* x,
                          int B, void* stream) {
  API_GUARD(plan);
  PINT_TRY(check_batch(B, u, x));
  Plan& p = plan->p;
  PINT_TRY(check_stepper(p, st));
  hipStream_t s = (hipStream_t)stream;
  const CnFactors* f = nullptr;
  PINT_TRY(cn_factors(p, st->dt, st->terms, s, &f));
  const size_t sd = (size_t)3 * p.ncoef * 2;
  for (int b0 = 0; b0 < B; b0 += p.max_batch) {
    const int nb = (B - b0) < p.max_batch ? (B - b0) : p.max_batch;
    PINT_TRY(sp_cn(p, *f, *st, nullptr, u + b0 * sd, x + b0 * sd, nb, s));
  }
  return PINT_OK;
}

pint_status pint_step(pint_plan* plan, const pint_stepper* st, const double* u_in, double* u_out,
                      int B, int nsteps, void* stream) {
  API_GUARD(plan);
  PINT_TRY(check_batch(B, u_in, u_out));
  PINT_TRY(check_stepper(plan->p, st));
  if (nsteps < 0) {
    set_error("nsteps must be >= 0");
    return PINT_E_INVAL;
  }
  return propagate(plan->p, *st, u_in, u_out, B, nsteps, (hipStream_t)stream);
}

pint_status pint_sl_steps(pint_plan* plan, const pint_sl_stepper* st, const double* u_prev,
                          const double* u, double* out, double* out_prev, int B, int nsteps,
                          void* stream) {
  API_GUARD(plan);
  if (!st) {
    set_error("null stepper");
    return PINT_E_INVAL;
  }
  return sl_steps(plan->p, *st, u_prev, u, out, out_prev, B, nsteps, (hipStream_t)stream);
}

// Parareal (Sec. 3.1) with an SL-SI-SETTLS coarse propagator (Sec. 2.3.2).
// The serial sweep is the coarsest level, where Sec. 3.2.4 runs the two-step
// scheme in every step: each slice's coarse run starts from the corrected
// U_n and the last-but-one state P_{n-1} of the previous slice's run (saved
// per slice in Pold), the very first step of the horizon in the one-step
// variant.  restart = 1 instead starts every slice's run in the one-step
// variant.  Iteration k leaves slices n < k untouched (they are converged),
// propagates slices k..N-1 of all instances with the fine IMEX steps as one
// batch and sweeps U_{n+1} = (G(U_n, P_{n-1}) - G_old_n) + F_n serially over
// n, the instances of a slice together (G and P at slice k are unchanged:
// their inputs are those of the previous sweep).  All on one stream.
// States are [slice][instance].
pint_status pint_parareal_sl(pint_plan* plan, const pint_stepper* fine, int fine_steps,
                             pint_plan* coarse_plan, const pint_sl_stepper* coarse,
                             int coarse_steps, int n_slices, int n_inst, int n_iter, int restart,
                             const double* u0, double* u_slices, void* stream) {
  API_GUARD(plan);
  if (!fine || !coarse || !u0 || !u_slices) {
    set_error("null argument");
    return PINT_E_INVAL;
  }
  Plan& p = plan->p;
  Plan& pc = coarse_plan ? coarse_plan->p : p;
  PINT_TRY(check_stepper(p, fine));
  if (fine_steps < 1 || coarse_steps < 1 || n_slices < 1 || n_inst < 1 || n_iter < 0 ||
      (restart != 0 && restart != 1)) {
    set_error("fine_steps, coarse_steps, n_slices, n_inst must be >= 1, n_iter >= 0 and "
              "restart 0 or 1");
    return PINT_E_INVAL;
  }
  if (pc.M > p.M || pc.a != p.a || pc.omega != p.omega || pc.phibar != p.phibar) {
    set_error("coarse plan must have M <= the fine M and the same planet and Phibar");
    return PINT_E_INVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const int N = n_slices, I = n_inst;
  const size_t sd = (size_t)3 * p.ncoef * 2, sdc = (size_t)3 * pc.ncoef * 2;
  const size_t ss = sd * I;                       // doubles per slice (all instances)
  const size_t ssc = sdc * I;                     // the same at the coarse truncation
  const size_t sb = ss * sizeof(double);
  const bool trunc = pc.M != p.M;
  DevBuf gold(p, kSlotPsGold), fv(p, kSlotPsFv), g(p, kSlotPsG), cin(p, kSlotPsCin),
      cout_(p, kSlotPsCout), pold(p, kSlotPsPold);
  PINT_TRY(gold.alloc(ss * N));
  PINT_TRY(fv.alloc(ss * N));
  PINT_TRY(g.alloc(ss));
  if (!restart) PINT_TRY(pold.alloc(ssc * N));
  if (trunc) {
    PINT_TRY(cin.alloc(ssc));
    PINT_TRY(cout_.alloc(ssc));
  }
  // G over slice n: x -> y for the I instances; the carried state enters
  // from slice n-1's Pold and slice n's leaves in Pold[n]
  auto G = [&](int n, const double* x, double* y) -> pint_status {
    const double* prev = (restart || n == 0) ? nullptr : pold.p + (size_t)(n - 1) * ssc;
    double* pout = restart ? nullptr : pold.p + (size_t)n * ssc;
    if (!trunc) return sl_steps(pc, *coarse, prev, x, y, pout, I, coarse_steps, s);
    PINT_TRY(spec_truncate(x, p.M, cin.p, pc.M, I, s));
    PINT_TRY(sl_steps(pc, *coarse, prev, cin.p, cout_.p, pout, I, coarse_steps, s));
    return spec_pad(cout_.p, pc.M, y, p.M, I, s);
  };
  double* U = u_slices;
  if (U != u0) PINT_HIP(hipMemcpyAsync(U, u0, sb, hipMemcpyDeviceToDevice, s));
  for (int n = 0; n < N; ++n) {
    PINT_TRY(G(n, U + n * ss, gold.p + n * ss));
    PINT_HIP(hipMemcpyAsync(U + (n + 1) * ss, gold.p + n * ss, sb, hipMemcpyDeviceToDevice, s));
  }
  for (int k = 0; k < n_iter && k < N; ++k) {
    PINT_TRY(propagate(p, *fine, U + k * ss, fv.p + k * ss, (N - k) * I, fine_steps, s));
    for (int n = k; n < N; ++n) {
      double* gn = gold.p + n * ss;
      if (n > k) {
        PINT_TRY(G(n, U + n * ss, g.p));
        PINT_TRY(pr_update(p, g.p, gn, fv.p + n * ss, U + (n + 1) * ss, ss, s));
        PINT_HIP(hipMemcpyAsync(gn, g.p, sb, hipMemcpyDeviceToDevice, s));
      } else {
        PINT_TRY(pr_update(p, gn, gn, fv.p + n * ss, U + (n + 1) * ss, ss, s));
      }
    }
  }
  return PINT_OK;
}

pint_status pint_solve(pint_plan* plan, const pint_pint_params* prm, const double* u0,
                       double* u_slices, pint_report* report, void* stream) {
  API_GUARD(plan);
  if (!u0 || !u_slices) {
    set_error("null state array");
    return PINT_E_INVAL;
  }
  return solve(plan->p, prm, u0, u_slices, report, (hipStream_t)stream);
}

pint_status pint_rel_diff(pint_plan* plan, const double* a, const double* c, double* out_host,
                          int B, void* stream) {
  API_GUARD(plan);
  PINT_TRY(check_batch(B, a, c));
  if (!out_host && B > 0) {
    set_error("null output");
    return PINT_E_INVAL;
  }
  return rel_diff(plan->p, a, c, out_host, B, (hipStream_t)stream);
}

pint_status pint_ke_spectrum(pint_plan* plan, const double* u, double* e, int B, void* stream) {
  API_GUARD(plan);
  PINT_TRY(check_batch(B, u, e));
  return ke_spectrum(plan->p, u, e, B, (hipStream_t)stream);
}

pint_status pint_spectral_errors(pint_plan* plan, const double* u, const double* ref, double* e,
                                 int B, void* stream) {
  API_GUARD(plan);
  PINT_TRY(check_batch(B, u, ref));
  PINT_TRY(check_batch(B, u, e));
  return spectral_errors(plan->p, u, ref, e, B, (hipStream_t)stream);
}

pint_status pint_grid_l2_errors(pint_plan* plan, const double* u, const double* ref,
                                double* out_host, int B, void* stream) {
  API_GUARD(plan);
  PINT_TRY(check_batch(B, u, ref));
  if (!out_host && B > 0) {
    set_error("null output");
    return PINT_E_INVAL;
  }
  return grid_l2_errors(plan->p, u, ref, out_host, B, (hipStream_t)stream);
}

pint_status pint_profile_enable(pint_plan* plan, unsigned kind_mask, int min_batch) {
  API_GUARD(plan);
  plan->p.prof_on = kind_mask != 0;
  plan->p.prof_mask = kind_mask;
  plan->p.prof_min_batch = min_batch;
  return PINT_OK;
}

pint_status pint_profile_read(pint_plan* plan, pint_prof_entry* out, int cap, int* n,
                              void* stream) {
  API_GUARD(plan);
  if (cap < 0) {
    set_error("cap must be >= 0");
    return PINT_E_INVAL;
  }
  return profile_read(plan->p, out, cap, n, (hipStream_t)stream);
}

const char* pint_last_error(void) { return last_error(); }

}  // extern "C"
