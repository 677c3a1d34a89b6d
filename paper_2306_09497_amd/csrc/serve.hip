// Serving engine: many Parareal / two-level MGRIT solves (Sec. 3) at once on
// one GPU with continuous batching.
//
// Every request runs the iteration of pint_solve as a state machine whose
// device work is either a propagation job (a contiguous range of the
// request's states advanced by a number of IMEX steps of one stepper) or a
// short host-issued update (Parareal correction, copies, increment norms).
// Each tick advances every pending job by one chunk of steps, and all jobs of
// one plan whose chunk has the same stepper and length run as ONE batched
// propagation: the fine propagations of different requests merge into common
// launches, and so do the serial coarse sweeps of different requests (each
// sweep step is a one-state job).  A job's chunks are fixed by its own step
// count and the server's steps_per_tick, never by the other jobs, and the
// propagator is batch invariant, so a request's result is bitwise the same
// alone and in any mix.
//
// Request state lives in one device arena allocated when the server is
// created (first-fit with coalescing); admission is by footprint, first in
// first out, so nothing is allocated in the serving loop.  Each plan's work
// goes to a stream of its own (plan 0: the caller's), so launches of
// different truncations overlap; a plan's workspace is only touched from its
// stream.
#include <algorithm>
#include <chrono>
#include <deque>
#include <map>
#include <math.h>
#include <memory>
#include <string.h>
#include <string>
#include <tuple>
#include <vector>

#include "pint_internal.h"

namespace pint {
namespace {

double clock_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// First-fit allocator over one device buffer, 256-byte granules.
class Arena {
 public:
  ~Arena() {
    if (base_) (void)hipFree(base_);
  }
  pint_status init(size_t bytes) {
    cap_ = round(bytes);
    if (hipMalloc(&base_, cap_) != hipSuccess) {
      base_ = nullptr;
      set_error("pint_server_create: hipMalloc of a %zu-byte arena failed", cap_);
      return PINT_E_NOMEM;
    }
    free_[0] = cap_;
    return PINT_OK;
  }
  size_t capacity() const { return cap_; }
  static size_t round(size_t b) { return (b + 255) & ~(size_t)255; }
  double* alloc(size_t bytes) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const size_t off = it->first, left = it->second - bytes;
      free_.erase(it);
      if (left) free_[off + bytes] = left;
      return reinterpret_cast<double*>(base_ + off);
    }
    return nullptr;
  }
  void release(double* p, size_t bytes) {
    bytes = round(bytes);
    size_t off = reinterpret_cast<char*>(p) - base_;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }

 private:
  char* base_ = nullptr;
  size_t cap_ = 0;
  std::map<size_t, size_t> free_;   // offset -> bytes
};

// count contiguous states: in -> out by `total` steps of st (in place after
// the first chunk)
struct Job {
  const double* in = nullptr;
  double* out = nullptr;
  int count = 0, total = 0, done = 0;
  pint_stepper st{};
};

enum Phase { kQueued, kInitSweep, kIterStart, kRelaxF, kRelaxG, kFine, kSweep, kIncr, kDone };

struct Request {
  long long id = 0;
  int plan = 0;
  pint_pint_params q{};
  const double* u0 = nullptr;
  double* out = nullptr;
  double t_submit = 0, t_start = 0, t_done = 0;
  size_t bytes = 0;
  double* mem = nullptr;
  double *U = nullptr, *Uprev = nullptr, *Fv = nullptr, *Gold = nullptr, *Gtmp = nullptr;
  Phase phase = kQueued;
  bool entered = false, job_active = false, finishing = false;
  int k = 0, n = 0, first = 0, relax_left = 0;
  Job job;
  int iters = 0;
  double incr = 0.0;
  long long fine_ss = 0, coarse_s = 0;
  pint_status status = PINT_OK;
  int state = PINT_REQ_QUEUED;
};

struct StepKey {
  double dt, nu;
  int q;
  unsigned terms;
  int chunk;
  bool operator<(const StepKey& o) const {
    return std::tie(dt, nu, q, terms, chunk) < std::tie(o.dt, o.nu, o.q, o.terms, o.chunk);
  }
};

}  // namespace
}  // namespace pint

using namespace pint;

struct pint_server {
  std::vector<Plan*> plans;
  std::vector<hipStream_t> streams;      // per plan: the caller's for plan 0
  std::vector<hipStream_t> owned;        // streams the server created
  Arena arena;
  int steps_per_tick = 1;
  int stage_states = 0;
  std::vector<double*> staging;          // per plan, stage_states states
  std::deque<Request*> queue;
  std::vector<Request*> active;
  std::map<long long, std::unique_ptr<Request>> all;
  long long next_id = 1;
  double t0 = 0;
  std::vector<double> incr;
  ~pint_server() {
    for (hipStream_t st : streams) (void)hipStreamSynchronize(st);
    for (double* p : staging)
      if (p) (void)hipFree(p);
    for (hipStream_t st : owned) (void)hipStreamDestroy(st);
  }
  double now() const { return clock_s() - t0; }
};

namespace pint {
namespace {

size_t state_doubles(const Plan& p) { return (size_t)3 * p.ncoef * 2; }

void start_job(Request& r, const pint_stepper& st, int steps, const double* in, double* out,
               int count) {
  r.job.in = in;
  r.job.out = out;
  r.job.count = count;
  r.job.total = steps;
  r.job.done = 0;
  r.job.st = st;
  r.job_active = true;
  r.entered = true;
}

void enter(Request& r, Phase ph) {
  r.phase = ph;
  r.entered = false;
}

pint_status copy(double* dst, const double* src, size_t doubles, hipStream_t s) {
  PINT_HIP(hipMemcpyAsync(dst, src, doubles * sizeof(double), hipMemcpyDeviceToDevice, s));
  return PINT_OK;
}

// Host steps of one request until it waits for a job or has finished.  The
// order of operations is that of pint_solve (two levels, same truncation).
pint_status run_machine(pint_server& S, Request& r) {
  Plan& p = *S.plans[r.plan];
  const pint_pint_params& q = r.q;
  const int N = q.n_intervals;
  const size_t sd = state_doubles(p);
  const bool mgrit = q.method == 1;
  hipStream_t s = S.streams[r.plan];
  auto finish = [&]() -> pint_status {
    PINT_TRY(copy(r.out, r.U, sd * (N + 1), s));
    r.finishing = true;
    r.phase = kDone;
    return PINT_OK;
  };
  while (!r.job_active && r.phase != kDone) {
    switch (r.phase) {
      case kQueued:
        return PINT_OK;
      case kInitSweep:   // iteration 0: U_{n+1} = G_n = phi_c(U_n)
        if (!r.entered) {
          start_job(r, q.coarse, q.coarse_steps, r.U + r.n * sd, r.Gold + r.n * sd, 1);
          break;
        }
        PINT_TRY(copy(r.U + (r.n + 1) * sd, r.Gold + r.n * sd, sd, s));
        r.coarse_s += q.coarse_steps;
        if (++r.n < N) {
          r.entered = false;
          continue;
        }
        enter(r, kIterStart);
        continue;
      case kIterStart:
        if (r.k >= q.max_iter) {
          PINT_TRY(finish());
          continue;
        }
        r.first = mgrit ? 0 : (r.k < N ? r.k : N);
        if (r.first >= N) {   // Parareal: every slice already exact
          PINT_TRY(finish());
          continue;
        }
        PINT_TRY(copy(r.Uprev, r.U, sd * (N + 1), s));
        r.relax_left = mgrit ? q.nrelax : 0;
        enter(r, r.relax_left > 0 ? kRelaxF : kFine);
        continue;
      case kRelaxF:      // CF pass: C-point i+1 <- Phi_0^m(C-point i)
        if (!r.entered) {
          start_job(r, q.fine, q.fine_steps, r.U, r.Fv, N);
          break;
        }
        PINT_TRY(copy(r.U + sd, r.Fv, sd * N, s));
        r.fine_ss += (long long)N * q.fine_steps;
        enter(r, --r.relax_left > 0 ? kRelaxF : kRelaxG);
        continue;
      case kRelaxG:      // coarse values Phi_1(v_i) of the relaxed C-points
        if (!r.entered) {
          start_job(r, q.coarse, q.coarse_steps, r.U, r.Gold, N);
          break;
        }
        r.coarse_s += (long long)N * q.coarse_steps;
        enter(r, kFine);
        continue;
      case kFine:        // the parallel part: F(U_n) of every active slice
        if (!r.entered) {
          start_job(r, q.fine, q.fine_steps, r.U + r.first * sd, r.Fv + r.first * sd,
                    N - r.first);
          break;
        }
        r.fine_ss += (long long)(N - r.first) * q.fine_steps;
        r.n = r.first;
        enter(r, kSweep);
        continue;
      case kSweep:       // U_{n+1} = (G(U_n^new) - G(U_n^old)) + F(U_n^old)
        if (r.n == r.first) {
          PINT_TRY(pr_update(p, r.Gold + r.n * sd, r.Gold + r.n * sd, r.Fv + r.n * sd,
                             r.U + (r.n + 1) * sd, sd, s));
        } else {
          if (!r.entered) {
            start_job(r, q.coarse, q.coarse_steps, r.U + r.n * sd, r.Gtmp, 1);
            break;
          }
          PINT_TRY(pr_update(p, r.Gtmp, r.Gold + r.n * sd, r.Fv + r.n * sd,
                             r.U + (r.n + 1) * sd, sd, s));
          PINT_TRY(copy(r.Gold + r.n * sd, r.Gtmp, sd, s));
          r.coarse_s += q.coarse_steps;
        }
        r.entered = false;
        if (++r.n == N) enter(r, kIncr);
        continue;
      case kIncr: {      // increments (synchronises the server stream)
        S.incr.resize((size_t)N * 4);
        PINT_TRY(rel_diff(p, r.U + sd, r.Uprev + sd, S.incr.data(), N, s));
        double worst = 0.0;
        bool bad = false;
        for (int i = 0; i < N; ++i)
          for (int f = 0; f < 4; ++f) {
            const double v = S.incr[(size_t)i * 4 + f];
            if (!isfinite(v)) bad = true;
            else if ((f == 0 || f == 3) && v > worst) worst = v;
          }
        r.iters = ++r.k;
        r.incr = bad ? NAN : worst;
        if (bad || worst > 1e6) {
          r.status = PINT_E_DIVERGED;
          PINT_TRY(finish());
          continue;
        }
        if (q.tol > 0.0 && worst <= q.tol) {
          PINT_TRY(finish());
          continue;
        }
        if (q.tol > 0.0 && r.k >= q.max_iter) r.status = PINT_E_NOTCONV;
        enter(r, kIterStart);
        continue;
      }
      case kDone:
        break;
    }
  }
  return PINT_OK;
}

// Admit queued requests in arrival order while their state fits the arena.
pint_status admit(pint_server& S) {
  while (!S.queue.empty()) {
    Request& r = *S.queue.front();
    double* mem = S.arena.alloc(r.bytes);
    if (!mem) break;
    S.queue.pop_front();
    Plan& p = *S.plans[r.plan];
    const size_t sd = state_doubles(p);
    const int N = r.q.n_intervals;
    r.mem = mem;
    r.U = mem;
    r.Uprev = r.U + sd * (N + 1);
    r.Fv = r.Uprev + sd * (N + 1);
    r.Gold = r.Fv + sd * N;
    r.Gtmp = r.Gold + sd * N;
    PINT_TRY(copy(r.U, r.u0, sd, S.streams[r.plan]));
    r.t_start = S.now();
    r.state = PINT_REQ_RUNNING;
    enter(r, kInitSweep);
    S.active.push_back(&r);
  }
  return PINT_OK;
}

// One chunk of `chunk` steps for every job in `jobs` (same plan and stepper).
pint_status run_group(pint_server& S, int pi, const std::vector<Job*>& jobs, int chunk) {
  Plan& p = *S.plans[pi];
  const size_t sd = state_doubles(p);
  const pint_stepper& st = jobs.front()->st;
  hipStream_t s = S.streams[pi];
  auto launch = [&](const double* in, double* out, int count) -> pint_status {
    for (int b0 = 0; b0 < count; b0 += p.max_batch) {
      const int nb = count - b0 < p.max_batch ? count - b0 : p.max_batch;
      PINT_TRY(imex_steps(p, st, in + b0 * sd, out + b0 * sd, nb, chunk, s));
    }
    return PINT_OK;
  };
  if (jobs.size() == 1) {
    Job& j = *jobs.front();
    return launch(j.done ? j.out : j.in, j.out, j.count);
  }
  // gather pieces of the jobs into the staging buffer, step, scatter back
  struct Piece {
    Job* j;
    int off, cnt, slot;
  };
  std::vector<Piece> seg;
  int used = 0;
  auto flush = [&]() -> pint_status {
    if (!used) return PINT_OK;
    double* stg = S.staging[pi];
    for (const Piece& c : seg) {
      const double* src = (c.j->done ? c.j->out : c.j->in) + (size_t)c.off * sd;
      PINT_TRY(copy(stg + (size_t)c.slot * sd, src, sd * c.cnt, s));
    }
    PINT_TRY(launch(stg, stg, used));
    for (const Piece& c : seg)
      PINT_TRY(copy(c.j->out + (size_t)c.off * sd, stg + (size_t)c.slot * sd, sd * c.cnt, s));
    seg.clear();
    used = 0;
    return PINT_OK;
  };
  for (Job* j : jobs) {
    int off = 0;
    while (off < j->count) {
      const int cnt = std::min(j->count - off, S.stage_states - used);
      seg.push_back({j, off, cnt, used});
      used += cnt;
      off += cnt;
      if (used == S.stage_states) PINT_TRY(flush());
    }
  }
  return flush();
}

pint_status tick(pint_server& S, int* pending) {
  PINT_TRY(admit(S));
  for (Request* r : S.active) PINT_TRY(run_machine(S, *r));
  // group the pending chunks per plan by (stepper, chunk length)
  std::vector<std::pair<Job*, int>> ran;
  for (int pi = 0; pi < (int)S.plans.size(); ++pi) {
    std::map<StepKey, std::vector<Job*>> groups;
    for (Request* r : S.active) {
      if (r->plan != pi || !r->job_active) continue;
      Job& j = r->job;
      const int chunk = std::min(S.steps_per_tick, j.total - j.done);
      groups[{j.st.dt, j.st.visc_nu, j.st.visc_order, j.st.terms, chunk}].push_back(&j);
    }
    for (auto& g : groups) {
      PINT_TRY(run_group(S, pi, g.second, g.first.chunk));
      for (Job* j : g.second) ran.push_back({j, g.first.chunk});
    }
  }
  for (hipStream_t st : S.streams) PINT_HIP(hipStreamSynchronize(st));
  for (auto& jr : ran) jr.first->done += jr.second;
  const double t = S.now();
  std::vector<Request*> still;
  for (Request* r : S.active) {
    if (r->job_active && r->job.done >= r->job.total) r->job_active = false;
    if (r->finishing) {   // its final copy has completed with the sync above
      r->t_done = t;
      r->state = r->status == PINT_E_DIVERGED ? PINT_REQ_FAILED : PINT_REQ_DONE;
      S.arena.release(r->mem, r->bytes);
      r->mem = nullptr;
      continue;
    }
    still.push_back(r);
  }
  S.active.swap(still);
  if (pending) *pending = (int)(S.active.size() + S.queue.size());
  return PINT_OK;
}

}  // namespace
}  // namespace pint

extern "C" {

pint_status pint_server_create(const pint_server_config* cfg, void* stream, pint_server** out) {
  if (!cfg || !out || cfg->n_plans < 1 || !cfg->plans || cfg->arena_bytes == 0 ||
      cfg->steps_per_tick < 1 || cfg->stage_states < 1) {
    set_error("pint_server_create: need a config with n_plans >= 1 plans, arena_bytes > 0, "
              "steps_per_tick >= 1, stage_states >= 1, and an output pointer");
    return PINT_E_INVAL;
  }
  for (int i = 0; i < cfg->n_plans; ++i)
    if (!cfg->plans[i]) {
      set_error("pint_server_create: plan %d is null", i);
      return PINT_E_INVAL;
    }
  std::unique_ptr<pint_server> S(new pint_server);
  for (int i = 0; i < cfg->n_plans; ++i) {
    hipStream_t st = (hipStream_t)stream;
    if (i > 0) {
      if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
        set_error("pint_server_create: hipStreamCreateWithFlags failed");
        return PINT_E_HIP;
      }
      S->owned.push_back(st);
    }
    S->streams.push_back(st);
  }
  S->steps_per_tick = cfg->steps_per_tick;
  S->stage_states = cfg->stage_states;
  S->t0 = clock_s();
  for (int i = 0; i < cfg->n_plans; ++i) {
    Plan& p = cfg->plans[i]->p;
    S->plans.push_back(&p);
    double* stg = nullptr;
    const size_t bytes = (size_t)cfg->stage_states * state_doubles(p) * sizeof(double);
    if (hipMalloc(&stg, bytes) != hipSuccess) {
      set_error("pint_server_create: hipMalloc of %zu staging bytes failed", bytes);
      return PINT_E_NOMEM;
    }
    S->staging.push_back(stg);
  }
  PINT_TRY(S->arena.init(cfg->arena_bytes));
  *out = S.release();
  return PINT_OK;
}

pint_status pint_server_destroy(pint_server* S) {
  if (!S) {
    set_error("null server");
    return PINT_E_INVAL;
  }
  delete S;
  return PINT_OK;
}

pint_status pint_server_submit(pint_server* S, const pint_request* req, long long* id) {
  if (!S || !req || !id) {
    set_error("null server, request or id");
    return PINT_E_INVAL;
  }
  if (req->plan < 0 || req->plan >= (int)S->plans.size()) {
    set_error("request plan index %d out of range [0, %zu)", req->plan, S->plans.size());
    return PINT_E_INVAL;
  }
  Plan& p = *S->plans[req->plan];
  const pint_pint_params& q = req->params;
  PINT_TRY(check_params(p, &q));
  if ((q.levels != 0 && q.levels != 2) || q.coarse_plan || q.resume || q.coarse_sl) {
    set_error("the server runs two-level solves on the plan's truncation "
              "(levels 2, no coarse_plan, resume 0)");
    return PINT_E_INVAL;
  }
  if (!req->u0 || !req->u_slices) {
    set_error("null u0 or u_slices");
    return PINT_E_INVAL;
  }
  // footprint: the driver scratch pint_solve needs for these parameters (the
  // same function as pint_plan_workspace_bytes) plus the request's own copy
  // of its slice states
  const int N = q.n_intervals;
  Footprint fp;
  PINT_TRY(solve_footprint(p, &q, fp, false));
  size_t scratch = 0;
  for (int i = 0; i < kSlotCount; ++i) scratch += fp.slot[i];
  const size_t bytes = (scratch + ((size_t)N + 1) * state_doubles(p)) * sizeof(double);
  if (Arena::round(bytes) > S->arena.capacity()) {
    set_error("request needs %zu bytes of state, the arena holds %zu", bytes,
              S->arena.capacity());
    return PINT_E_NOMEM;
  }
  // Crank-Nicolson factors of both steppers now, not in the serving loop
  const CnFactors* f = nullptr;
  PINT_TRY(cn_factors(p, q.fine.dt, q.fine.terms, S->streams[req->plan], &f));
  PINT_TRY(cn_factors(p, q.coarse.dt, q.coarse.terms, S->streams[req->plan], &f));
  std::unique_ptr<Request> r(new Request);
  r->id = S->next_id++;
  r->plan = req->plan;
  r->q = q;
  r->u0 = req->u0;
  r->out = req->u_slices;
  r->bytes = bytes;
  r->t_submit = S->now();
  *id = r->id;
  S->queue.push_back(r.get());
  S->all[r->id] = std::move(r);
  return PINT_OK;
}

pint_status pint_server_tick(pint_server* S, int* pending) {
  if (!S) {
    set_error("null server");
    return PINT_E_INVAL;
  }
  return tick(*S, pending);
}

pint_status pint_server_status(pint_server* S, long long id, pint_request_status* st) {
  if (!S || !st) {
    set_error("null server or status");
    return PINT_E_INVAL;
  }
  auto it = S->all.find(id);
  if (it == S->all.end()) {
    set_error("unknown request id %lld", id);
    return PINT_E_INVAL;
  }
  const Request& r = *it->second;
  st->state = r.state;
  st->status = r.status;
  st->iters = r.iters;
  st->incr = r.incr;
  st->t_submit = r.t_submit;
  st->t_start = r.t_start;
  st->t_done = r.t_done;
  st->fine_slice_steps = r.fine_ss;
  st->coarse_steps = r.coarse_s;
  return PINT_OK;
}

pint_status pint_server_clock(pint_server* S, double* t) {
  if (!S || !t) {
    set_error("null server or output");
    return PINT_E_INVAL;
  }
  *t = S->now();
  return PINT_OK;
}

}  // extern "C"
