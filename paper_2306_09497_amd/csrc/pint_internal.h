// Internal declarations of the MI355X shallow-water propagator library.
//
// Index spaces used by the kernels (M = truncation, nlat2 = nlat / 2):
//  * packed coefficient index  idx(m,n) = m(2M+3-m)/2 + (n-m), n <= M
//  * "row space": every (m, n) with n <= M+1 (one extra degree needed by the
//    vector transforms), grouped per zonal wavenumber m and per parity
//    p = (n-m) mod 2: row = rowoff[2m+p] + (n-m-p)/2.  The Legendre table,
//    the synthesis inputs and the analysis outputs all live in row space, so
//    every (m, p) block is one dense GEMM operand.
//  * work layout of a batch of B states: element (idx, b, field) at
//    ((idx*B + b)*3 + field) complex, i.e. batch innermost, so that one
//    (m, n) row of the GEMM operands is contiguous across the batch.
//  * GEMM column c = (b*nf + f)*2 + reim, nf = 6 fields in synthesis
//    (xi, delta, Phi', G, U, V) and 4 in analysis (N_Phi, K, A, B).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pint.h"
#include "device_common.h"

namespace pint {

constexpr int kMaxSweepChunks = 64;  // fine-propagation chunks per PinT iteration

void set_error(const char* fmt, ...);

#define PINT_HIP(call)                                                        \
  do {                                                                        \
    hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess) {                                                   \
      ::pint::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                        __FILE__, __LINE__);                                  \
      return PINT_E_HIP;                                                      \
    }                                                                         \
  } while (0)

// Return the status of a library call that failed.
#define PINT_TRY(x)                  \
  do {                               \
    pint_status st_ = (x);           \
    if (st_ != PINT_OK) return st_;  \
  } while (0)

// LU factors of the two tridiagonal chains of (I - dt/4 L) per m, for one
// (dt, terms), as the coefficients of the two first-order recurrences
//   y_i = alph_i y_{i-1} + invpiv_i r_i,   x_i = gam_i x_{i+1} + y_i
// (alph_i = -l_i / piv_i, gam_i = -u_i / piv_i); [2 chains][ncoef] each.
struct CnFactors {
  double2* alph = nullptr;
  double2* gam = nullptr;
  double2* invpiv = nullptr;
};

struct GemmTiles {       // (problem, row tile) list of one ragged batched GEMM
  int* dev = nullptr;    // int2 {problem p = 2m+par, row0} per row tile
  int count = 0;
};

enum ProfKind {
  PK_PREP = 0, PK_SYNTH, PK_RING, PK_ANAL, PK_ASSEMBLE, PK_CN, PK_LAYOUT, PK_PINT, PK_SRING,
  PK_SL, PK_COUNT
};

struct ProfRec {
  int kind, batch;
  hipEvent_t a, b;
};

struct Plan {
  int M, nlon, nlat, nlat2, ncoef, nrows, max_batch;
  int prec = PINT_FP64;        // PINT_FP64 or PINT_LEG_FP32 (transforms in FP32)
  double a, omega, g, phibar;
  // device tables
  double* mu = nullptr;        // [nlat] north to south
  double* w = nullptr;         // [nlat]
  double* c2 = nullptr;        // [nlat] 1 - mu^2 (= sin^2 colatitude)
  double* ptab = nullptr;      // [nrows][nlat2] Pbar_n^m(mu_j), north half
  double* ptabT = nullptr;     // [nlat2][nrows] the same table transposed (analysis GEMM)
  float* ptab32 = nullptr;     // FP32 copies of both (PINT_LEG_FP32 only)
  float* ptabT32 = nullptr;
  int* rowoff = nullptr;       // [2(M+1)+1] device copy
  int* rowinfo = nullptr;      // [nrows] packed (m << 16 | n)
  int* coefmn = nullptr;       // [ncoef] packed (m << 16 | n)
  double2* twid = nullptr;     // [nlon] exp(-2 pi i t / nlon)
  float2* twid32 = nullptr;    // the same in FP32
  double4* cnco = nullptr;     // [ncoef] linear-operator coefficients (A/W, B/W, C/W, n(n+1)/a^2)
  std::vector<int> h_rowoff;   // host copy
  GemmTiles syn_tiles, ana_tiles;
  // spectral kernel tasks: chains (zonal wavenumbers) of one state packed
  // onto the lanes of one wave, kSpecTaskInts ints per task
  int* spec_tasks = nullptr;
  int n_spec_tasks = 0;
  // workspace (sized for max_batch)
  // GEMM and ring workspace, sized for FP64; FP32 in PINT_LEG_FP32 mode
  double* S = nullptr;         // [nrows][12 B]   synthesis GEMM input
  double* F = nullptr;         // [(M+1) nlat][12 B] synthesis output (Fourier coefficients)
  double* G = nullptr;         // [(M+1) nlat][8 B] ring output
  double* Q = nullptr;         // [nrows][8 B]    analysis output
  double* Ua = nullptr;        // states [B][3][ncoef] complex: first half-step result
  double* N1 = nullptr;        //   and first-stage tendencies of the IMEX step
  // serial correction sweep of the PinT drivers: a B = 1 workspace and a
  // stream of its own, so that the sweep runs beside the fine propagation of
  // later slices (chunks released by events)
  struct Work {
    double *S = nullptr, *F = nullptr, *G = nullptr, *Q = nullptr, *Ua = nullptr, *N1 = nullptr;
  } side;
  hipStream_t side_stream = nullptr;
  hipStream_t capture_stream = nullptr;  // PinT iterations are captured on it
  bool use_graphs = true;                // replay repeating iterations from a graph
  std::vector<hipEvent_t> chunk_ev;  // one per fine-propagation chunk
  hipEvent_t join_ev = nullptr;      // end of a sweep on side_stream
  // the next iteration's relaxation runs on relax_stream beside the sweep
  // (two-level MGRIT, one CF pass): relax_ev[c] releases its chunk c,
  // relax_done_ev[c] marks it done, relax_join_ev ends the relax stream's work
  hipStream_t relax_stream = nullptr;
  std::vector<hipEvent_t> relax_ev, relax_done_ev;
  hipEvent_t relax_join_ev = nullptr;
  bool pipeline_relax = true;
  int sweep_chunks = 4;
  double* red = nullptr;       // reduction scratch
  double* diag = nullptr;      // L2-error partial sums [3 max_batch][nlat][2]
  double* h_red = nullptr;     // pinned host mirror
  double* h_incr = nullptr;    // pinned host staging of the PinT increments
  size_t h_incr_n = 0;         //   (doubles), grown on demand
  double* sl_lat = nullptr;    // [nlat + 4] latitudes extended across the poles (SL)
  size_t ws_bytes = 0;         // device bytes held: tables, workspace, factors, pool
  size_t base_bytes = 0;       // of which made at creation
  long long n_allocs = 0;      // device allocations made since creation
  // timing events of the PinT phases (iteration start, fine propagation
  // done, serial coarse part done)
  hipEvent_t ph_ev[3] = {nullptr, nullptr, nullptr};
  // Legendre GEMM launch shape per (synthesis / analysis, small / large
  // launch class), set by the autotuner; and the tuned time per launch
  int gemm_variant[2][2] = {{0, 0}, {0, 0}};
  float gemm_tuned_ms[2][2] = {{0.0f, 0.0f}, {0.0f, 0.0f}};
  // ring workgroup size per launch class (few / many states): variant 0 is
  // 256 threads for few states and 128 for many, variant 1 the other one
  int ring_variant[2] = {0, 0};
  float ring_tuned_ms[2] = {0.0f, 0.0f};
  // device scratch of the PinT drivers, kept between calls and grown on
  // demand (slot -> buffer, doubles)
  std::vector<std::pair<double*, size_t>> pool;
  std::map<std::pair<double, unsigned>, CnFactors> cn_cache;
  // kernel timing (pint_profile_enable)
  bool prof_on = false;
  unsigned prof_mask = 0;
  int prof_min_batch = 0;
  std::vector<ProfRec> prof;       // launches recorded since the last read
  std::vector<hipEvent_t> ev_pool; // reusable events
  size_t prof_used = 0;
};

// While in scope, kernels enqueued on the plan use its B = 1 sweep workspace
// (enqueueing is sequential on the host, so each launch captures the
// pointers current at its enqueue).
struct SideWork {
  Plan& p;
  explicit SideWork(Plan& pl) : p(pl) { swap(); }
  ~SideWork() { swap(); }
  void swap() {
    std::swap(p.S, p.side.S);
    std::swap(p.F, p.side.F);
    std::swap(p.G, p.side.G);
    std::swap(p.Q, p.side.Q);
    std::swap(p.Ua, p.side.Ua);
    std::swap(p.N1, p.side.N1);
  }
};

// Bracket one kernel launch with events when profiling is enabled.
int prof_begin(Plan& p, int kind, int batch, hipStream_t s);
pint_status profile_read(Plan& p, pint_prof_entry* out, int cap, int* n, hipStream_t s);
void prof_end(Plan& p, int rec, hipStream_t s);

struct ProfScope {
  Plan& p;
  hipStream_t s;
  int rec;
  ProfScope(Plan& pl, int kind, int batch, hipStream_t st) : p(pl), s(st) {
    const int nb = batch < 0 ? -batch : batch;
    rec = (pl.prof_on && ((pl.prof_mask >> kind) & 1u) && nb >= pl.prof_min_batch)
              ? prof_begin(pl, kind, batch, st)
              : -1;
  }
  ~ProfScope() {
    if (rec >= 0) prof_end(p, rec, s);
  }
};

const char* last_error();
pint_status create(const pint_config* cfg, hipStream_t s, pint_plan** out);
void destroy(pint_plan* pp);

// ---- kernels / launchers (each returns PINT_OK or an error) ----
pint_status build_tables(Plan& p, hipStream_t s);
pint_status cn_factors(Plan& p, double dt, unsigned terms, hipStream_t s, const CnFactors** out);
pint_status cn_factors_fill(const Plan& p, double dt, unsigned terms, const CnFactors& f,
                            hipStream_t s);
// the library's static scratch of the current device (set up at plan creation)
pint_status noalloc_init_device();

// Spectral kernels on public-layout states (one wave per (m, state)):
//  sp_cn_prep  Ua = CN(in) (no viscosity); S = synthesis input of Ua
//  sp_stage1   N1 = N(Q); S = synthesis input of Ua + dt N1
//  sp_stage2   U = D_nu CN(Ua + dt/2 (N1 + N(Q))); chain: Ua = CN(U), S from
//              Ua (the next step begins); else out = U
//  sp_prep     S = synthesis input of in;  sp_tend  out = N(Q)
//  sp_cn       out = CN(in) with st0 (and its viscosity); with st1, st0's
//              half step without viscosity then st1's with it
pint_status sp_cn_prep(Plan& p, const CnFactors& f, const pint_stepper& st, const double* in,
                       int B, hipStream_t s);
pint_status sp_stage1(Plan& p, double dt, int B, hipStream_t s);
pint_status sp_stage2(Plan& p, const CnFactors& f, const pint_stepper& st, double* out,
                      bool chain, int B, hipStream_t s, const double* cf = nullptr,
                      double* corr = nullptr);
pint_status sp_prep(Plan& p, const double* in, int B, hipStream_t s);
pint_status sp_tend(Plan& p, double* out, int B, hipStream_t s);
pint_status sp_cn(Plan& p, const CnFactors& f, const pint_stepper& st0, const pint_stepper* st1,
                  const double* in, double* out, int B, hipStream_t s);
// nsteps IMEX steps of B <= max_batch public-layout states (out may alias in)
// argument checks of the public entry points (PINT_E_INVAL with a message)
pint_status check_stepper(const Plan& p, const pint_stepper* st);
pint_status check_params(const Plan& p, const pint_pint_params* q);
// With corr (needs nsteps >= 1 and the nonlinear term): out holds G_old on
// entry and receives the result G, and corr = (G - G_old) + cf (a PinT
// correction fused into the last step); chain_out: the last kernel also
// makes the first half step of corr (the next sweep step), which a call
// with prepped = true then starts from instead of `in`.
// given: use this factor set instead of the plan's cached one.
pint_status imex_steps(Plan& p, const pint_stepper& st, const double* in, double* out, int B,
                       int nsteps, hipStream_t s, const double* cf = nullptr,
                       double* corr = nullptr, bool prepped = false, bool chain_out = false,
                       const CnFactors* given = nullptr);

// transforms on the GEMM workspace
// prec: PINT_FP64 (also used by the public scalar transforms) or PINT_LEG_FP32
pint_status spec_truncate(const double* in, int Mf, double* out, int Mc, int B, hipStream_t s);
pint_status spec_pad(const double* in, int Mc, double* out, int Mf, int B, hipStream_t s);
pint_status legendre_synth(Plan& p, int B, int nf, int prec, hipStream_t s);
pint_status legendre_anal(Plan& p, int B, int nf, int prec, hipStream_t s);
// time the launch shapes of both Legendre transforms and of the ring kernel
// at states[0] (small launch class) and states[1] (large) states per launch,
// keep the fastest
pint_status tune_legendre(Plan& p, const int (&states)[2], hipStream_t s);
// Packs the chains m = 0..M of one state onto waves for the spectral
// kernels (a function of M only) and uploads the task table.
pint_status spec_tasks_build(Plan& p, size_t* total);
pint_status tune_ring(Plan& p, const int (&states)[2], hipStream_t s);
pint_status ring_tendency(Plan& p, int B, hipStream_t s);
bool ring_supported(int nlon);
size_t ring_lds_bytes(int nlon, int prec);
pint_status ring_prepare(int nlon);

// scalar transforms (public layout)
pint_status scalar_synthesis(Plan& p, const double* spec, double* grid, int B, hipStream_t s);
pint_status scalar_analysis(Plan& p, const double* grid, double* spec, int B, hipStream_t s);

// elementwise helpers (public layout, n doubles)
pint_status pr_update(Plan& p, const double* gnew, const double* gold, const double* f,
                      double* out, size_t n, hipStream_t s);
pint_status rel_diff(Plan& p, const double* a, const double* c, double* out_host, int B,
                     hipStream_t s);
pint_status rel_diff_enqueue(Plan& p, const double* a, const double* c, double* dev,
                             double* host, int B, hipStream_t s);
void rel_diff_finish(const double* host, double* out_host, int B);

// diagnostics (Sec. 5, Sec. 5.1): KE spectrum [B][M+1] and spectral max-norm
// errors [B][3][M+1] on the device, physical-space L2 errors [B][3] to the host
pint_status ke_spectrum(Plan& p, const double* u, double* e, int B, hipStream_t s);
pint_status spectral_errors(Plan& p, const double* u, const double* ref, double* e, int B,
                            hipStream_t s);
pint_status grid_l2_errors(Plan& p, const double* u, const double* ref, double* out_host, int B,
                           hipStream_t s);
// sums of squares over each ring of nspec / 2 synthesised pairs held in F:
// part[pair][latitude][2]
pint_status ring_sumsq(Plan& p, int nspec, double* part, hipStream_t s);

// Device scratch kept in the plan between calls, grown on demand.
struct DevBuf {
  Plan& pl;
  int slot;
  double* p = nullptr;
  DevBuf(Plan& plan, int s) : pl(plan), slot(s) {}
  pint_status alloc(size_t n) {
    if (pl.pool.size() <= (size_t)slot) pl.pool.resize(slot + 1, {nullptr, 0});
    auto& b = pl.pool[slot];
    if (b.second < n) {
      if (b.first) (void)hipFree(b.first);
      pl.ws_bytes -= b.second * sizeof(double);
      b = {nullptr, 0};
      ++pl.n_allocs;
      if (hipMalloc(&b.first, n * sizeof(double)) != hipSuccess) {
        b.first = nullptr;
        set_error("hipMalloc(%zu bytes) of solver scratch failed", n * sizeof(double));
        return PINT_E_NOMEM;
      }
      b.second = n;
      pl.ws_bytes += n * sizeof(double);
    }
    p = b.first;
    return PINT_OK;
  }
};
enum PoolSlot { kSlotGold, kSlotFv, kSlotUprev, kSlotGtmp, kSlotCin, kSlotCinSide, kSlotW,
                kSlotFl, kSlotGl, kSlotTmp, kSlotF2, kSlotG2, kSlotGz, kSlotSlGrid, kSlotSlF,
                kSlotSlO, kSlotPsGold, kSlotPsFv, kSlotPsG, kSlotPsCin, kSlotPsCout,
                kSlotPsPrev, kSlotPsPold, kSlotIncr, kSlotFvR, kSlotRS, kSlotRF, kSlotRG,
                kSlotRQ, kSlotRUa, kSlotRN1, kSlotCount };

// Device memory a workload needs on one plan: doubles per pool slot and the
// Crank-Nicolson factor keys (dt, terms) it uses.  Filled by the drivers'
// footprint functions; reserve() allocates exactly this.
struct Footprint {
  size_t slot[kSlotCount] = {};
  std::vector<std::pair<double, unsigned>> cn;        // on the plan itself
  std::vector<std::pair<double, unsigned>> cn_coarse; // on the coarse plan
  size_t host_doubles = 0;                            // pinned host staging
  void need(int s, size_t n) {
    if (n > slot[s]) slot[s] = n;
  }
  void factors(std::vector<std::pair<double, unsigned>>& v, double dt, unsigned terms) {
    const auto k = std::make_pair(dt, terms & (PINT_T_LG | PINT_T_LC));
    for (const auto& e : v)
      if (e == k) return;
    v.push_back(k);
  }
};
size_t cn_factor_bytes(const Plan& p);
// footprint of pint_solve(q) (q may be NULL) and of pint_sl_steps with
// stepper sl (may be NULL) on plan p
// (pipelined: with the buffers of the relaxation pipelined beside the sweep
// when the solve uses it; the server does not)
pint_status solve_footprint(const Plan& p, const pint_pint_params* q, Footprint& fp,
                            bool pipelined = true);
void sl_footprint(const Plan& p, const pint_sl_stepper& st, Footprint& fp);
pint_status sl_check(const Plan& p, const pint_sl_stepper& st, int B, int nsteps);
size_t footprint_bytes(const Plan& p, const Plan* pc, const Footprint& fp);
pint_status reserve(Plan& p, Plan* pc, const Footprint& fp, hipStream_t s);


// Semi-Lagrangian SETTLS steps (Sec. 2.3.2; one-step variant, Sec. 3.2.4)
pint_status ring_sl_grid(Plan& p, double* grid, int Bt, hipStream_t s);
pint_status ring_sl_anal(Plan& p, const double* grid, int B, hipStream_t s);
pint_status sp_sl_solve(Plan& p, const CnFactors& f, double dt, int visc_order, double visc_nu,
                        double* out, int B, hipStream_t s);
pint_status sl_steps(Plan& p, const pint_sl_stepper& st, const double* u_prev, const double* u,
                     double* out, double* out_prev, int B, int nsteps, hipStream_t s);

}  // namespace pint

struct pint_plan {
  pint::Plan p;
};
