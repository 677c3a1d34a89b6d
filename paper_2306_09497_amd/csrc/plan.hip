// Plan creation: validation, index tables, device-generated FP64 tables
// (Gauss nodes/weights, normalised associated Legendre functions, FFT
// twiddles), Crank-Nicolson tridiagonal factors, and the workspace.
#include <math.h>
#include <algorithm>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "pint_internal.h"

namespace pint {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

const char* last_error() { return g_err; }

// ---------------------------------------------------------------------------
// Gauss-Legendre nodes (Sec. 2.2 Gauss grid).  Newton iteration on
// P_nlat(cos theta) in the colatitude theta.  Near the poles x = cos(theta)
// cannot locate the root to full relative precision, so P_n is evaluated
// from d = 1 - x = 2 sin^2(theta/2) with the difference form of the
// three-term recurrence,
//   D_k = P_k - P_{k-1} = ((k-1) D_{k-1} - (2k-1) d P_{k-1}) / k,
// and x P_n - P_{n-1} = D_n - d P_n, so that
//   dP_n/dtheta = n (D_n - d P_n) / sin(theta),
//   w = 2 / ((1-x^2) P_n'(x)^2) = 2 sin^2(theta) / (n (D_n - d P_n))^2,
// and 1 - mu^2 = sin^2(theta), all without cancellation.  One thread per
// northern node; the southern node is its mirror.
// ---------------------------------------------------------------------------
__device__ inline void legendre_theta(int n, double th, double* pn, double* dn, double* d) {
  const double sh = sin(0.5 * th);
  const double dd = 2.0 * sh * sh;
  double p1 = 1.0 - dd, D = -dd;       // P_1, P_1 - P_0
  for (int k = 2; k <= n; ++k) {
    D = ((k - 1.0) * D - (2.0 * k - 1.0) * dd * p1) / k;
    p1 += D;
  }
  *pn = p1;
  *dn = D;
  *d = dd;
}

__global__ void k_gauss(int nlat, double* mu, double* w, double* c2) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int nh = nlat / 2;
  if (j >= nh) return;
  const double n = (double)nlat;
  double th = M_PI * (j + 0.75) / (n + 0.5);
  double pn, dn, d;
  for (int it = 0; it < 16; ++it) {
    legendre_theta(nlat, th, &pn, &dn, &d);
    const double dth = pn * sin(th) / (n * (dn - d * pn));
    th -= dth;
    if (fabs(dth) < 1e-18 * th) break;
  }
  legendre_theta(nlat, th, &pn, &dn, &d);
  const double s = sin(th);
  const double q = n * (dn - d * pn);
  const double wj = 2.0 * s * s / (q * q);
  const double x = cos(th);
  mu[j] = x;
  mu[nlat - 1 - j] = -x;
  w[j] = wj;
  w[nlat - 1 - j] = wj;
  c2[j] = s * s;
  c2[nlat - 1 - j] = s * s;
}

// Normalised associated Legendre functions Pbar_n^m(mu_j), n = m..M+1, on the
// northern nodes, written in row space.  Recurrences:
//   Pbar_0^0 = 1,  Pbar_m^m = sqrt((2m+1)/(2m)) sqrt(1-mu^2) Pbar_{m-1}^{m-1},
//   Pbar_{m+1}^m = sqrt(2m+3) mu Pbar_m^m,
//   Pbar_n^m = (mu Pbar_{n-1}^m - eps_{n-1}^m Pbar_{n-2}^m) / eps_n^m,
//   eps_n^m = sqrt((n^2 - m^2) / (4 n^2 - 1)).
__global__ void k_ptab(int M, int nlat2, int nrows, const double* mu, const double* c2,
                       const int* rowoff, double* ptab, double* ptabT) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  const int m = blockIdx.y;
  if (j >= nlat2) return;
  const double x = mu[j];
  const double s = sqrt(c2[j]);
  double pmm = 1.0;
  for (int k = 1; k <= m; ++k) pmm *= sqrt((2.0 * k + 1.0) / (2.0 * k)) * s;
  const int o0 = rowoff[2 * m], o1 = rowoff[2 * m + 1];
  double pprev = pmm;                  // n - 2
  double pcur = sqrt(2.0 * m + 3.0) * x * pmm;  // n - 1 (= m + 1)
  ptab[(size_t)o0 * nlat2 + j] = pmm;
  ptabT[(size_t)j * nrows + o0] = pmm;
  if (m + 1 <= M + 1) {
    ptab[(size_t)o1 * nlat2 + j] = pcur;
    ptabT[(size_t)j * nrows + o1] = pcur;
  }
  for (int n = m + 2; n <= M + 1; ++n) {
    const double e1 = sqrt(((double)(n - 1) * (n - 1) - (double)m * m) /
                           (4.0 * (n - 1) * (n - 1) - 1.0));
    const double e0 = sqrt(((double)n * n - (double)m * m) / (4.0 * n * n - 1.0));
    const double pn = (x * pcur - e1 * pprev) / e0;
    const int par = (n - m) & 1;
    const int row = (par ? o1 : o0) + ((n - m - par) >> 1);
    ptab[(size_t)row * nlat2 + j] = pn;
    ptabT[(size_t)j * nrows + row] = pn;
    pprev = pcur;
    pcur = pn;
  }
}

// FP32 copies (round to nearest) of the FP64 tables for PINT_LEG_FP32.
__global__ void k_to_float(const double* __restrict__ x, float* __restrict__ y, size_t n) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = (float)x[t];
}

__global__ void k_twiddle(int nlon, double2* tw) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nlon) return;
  double sn, cs;
  sincospi(2.0 * t / nlon, &sn, &cs);
  tw[t] = make_double2(cs, -sn);      // exp(-2 pi i t / nlon)
}

// Per-coefficient linear-operator coefficients of the chain form (see
// cn_factors), with the Coriolis factor W = 2 Omega divided out.
__global__ void k_cn_coef(int M, int ncoef, double a, const int* coefmn, double4* co) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= ncoef) return;
  const int m = coefmn[i] >> 16, n = coefmn[i] & 0xffff;
  const CnCoef c = cn_coef(m, n, M, a, 1.0, true);
  co[i] = make_double4(c.A, c.B, c.C, c.lap);
}

// Latitudes of the Gauss rows extended by two mirrored rows beyond each pole
// (the semi-Lagrangian interpolation stencil crosses the poles): entry j + 2
// is asin(mu_j); the rows beyond the north pole are pi - lat of the first
// rows, those beyond the south pole -pi - lat of the last rows.
__global__ void k_sl_lat(int nlat, const double* mu, double* lat) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nlat + 4) return;
  const double pi = 3.14159265358979323846264338328;
  double v;
  if (i == 0) v = pi - asin(mu[1]);
  else if (i == 1) v = pi - asin(mu[0]);
  else if (i == nlat + 2) v = -pi - asin(mu[nlat - 1]);
  else if (i == nlat + 3) v = -pi - asin(mu[nlat - 2]);
  else v = asin(mu[i - 2]);
  lat[i] = v;
}

template <typename T>
static pint_status dalloc(T** ptr, size_t count, size_t* total) {
  void* v = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&v, count * sizeof(T));
  if (e != hipSuccess) {
    set_error("hipMalloc(%zu bytes) failed: %s", count * sizeof(T), hipGetErrorString(e));
    return PINT_E_NOMEM;
  }
  *ptr = (T*)v;
  if (total) *total += count * sizeof(T);
  return PINT_OK;
}

static void free_plan(Plan& p) {
  void* ptrs[] = {p.mu, p.w, p.c2, p.ptab, p.ptabT, p.ptab32, p.ptabT32, p.twid32,
                  p.rowoff, p.rowinfo, p.coefmn, p.twid, p.cnco, p.syn_tiles.dev,
                  p.ana_tiles.dev, p.S, p.F, p.G, p.Q, p.Ua, p.N1, p.red, p.diag,
                  p.side.S, p.side.F, p.side.G, p.side.Q, p.side.Ua, p.side.N1, p.sl_lat,
                  p.spec_tasks};
  for (void* q : ptrs)
    if (q) (void)hipFree(q);
  for (auto& b : p.pool)
    if (b.first) (void)hipFree(b.first);
  p.pool.clear();
  for (hipEvent_t e : p.chunk_ev) (void)hipEventDestroy(e);
  p.chunk_ev.clear();
  for (hipEvent_t e : p.relax_ev) (void)hipEventDestroy(e);
  p.relax_ev.clear();
  for (hipEvent_t e : p.relax_done_ev) (void)hipEventDestroy(e);
  p.relax_done_ev.clear();
  if (p.relax_join_ev) (void)hipEventDestroy(p.relax_join_ev);
  p.relax_join_ev = nullptr;
  if (p.relax_stream) (void)hipStreamDestroy(p.relax_stream);
  p.relax_stream = nullptr;
  if (p.join_ev) (void)hipEventDestroy(p.join_ev);
  p.join_ev = nullptr;
  for (hipEvent_t& e : p.ph_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  if (p.side_stream) (void)hipStreamDestroy(p.side_stream);
  p.side_stream = nullptr;
  if (p.capture_stream) (void)hipStreamDestroy(p.capture_stream);
  p.capture_stream = nullptr;
  if (p.h_red) (void)hipHostFree(p.h_red);
  if (p.h_incr) (void)hipHostFree(p.h_incr);
  for (hipEvent_t e : p.ev_pool) (void)hipEventDestroy(e);
  p.ev_pool.clear();
  for (auto& kv : p.cn_cache) {
    (void)hipFree(kv.second.alph);
    (void)hipFree(kv.second.gam);
    (void)hipFree(kv.second.invpiv);
  }
  p.cn_cache.clear();
}

static pint_status build_tiles(const std::vector<int>& rowoff, int M, int nlat2, bool synth,
                               int TR, GemmTiles* t, size_t* total) {
  // Tiles ordered by (m mod 8, m, parity, row): the kernels hand each XCD a
  // contiguous range of tiles, and work per tile falls with m, so grouping
  // m by residue mod 8 gives every XCD a near-equal share.
  std::vector<int> h;
  for (int cls = 0; cls < kNumXcd; ++cls) {
    for (int m = cls; m <= M; m += kNumXcd) {
      // a tile covers both parities of m (listed as p = 2m): synthesis tiles
      // run over the latitudes, analysis tiles over the longer parity's rows
      for (int par = 0; par < 1; ++par) {
        const int p = 2 * m + par;
        const int cnt = std::max(rowoff[p + 1] - rowoff[p], rowoff[p + 2] - rowoff[p + 1]);
        const int R = synth ? nlat2 : cnt;
        if (cnt == 0) continue;
        for (int r0 = 0; r0 < R; r0 += TR) {
          h.push_back(p);
          h.push_back(r0);
        }
      }
    }
  }
  t->count = (int)h.size() / 2;
  PINT_TRY(dalloc(&t->dev, h.size(), total));
  PINT_HIP(hipMemcpy(t->dev, h.data(), h.size() * sizeof(int), hipMemcpyHostToDevice));
  return PINT_OK;
}

pint_status create(const pint_config* cfg, hipStream_t s, pint_plan** out) {
  if (!cfg || !out) {
    set_error("pint_plan_create: null argument");
    return PINT_E_INVAL;
  }
  *out = nullptr;
  const int M = cfg->M, nlon = cfg->nlon, nlat = cfg->nlat;
  if (M < 1 || nlat < M + 2 || (nlat & 1) || nlon < 2 * M + 2 || nlon > kMaxNlon) {
    set_error("pint_plan_create: need M >= 1, even nlat >= M+2, 2M+2 <= nlon <= %d "
              "(got M=%d nlon=%d nlat=%d)", kMaxNlon, M, nlon, nlat);
    return PINT_E_INVAL;
  }
  if (M + 2 > 32767) {
    set_error("pint_plan_create: M too large");
    return PINT_E_INVAL;
  }
  if (!ring_supported(nlon)) {
    set_error("pint_plan_create: nlon=%d has no compiled ring FFT (supported: 64 96 128 192 "
              "256 384 512 640 768 1024)", nlon);
    return PINT_E_INVAL;
  }
  if (cfg->precision != PINT_FP64 && cfg->precision != PINT_LEG_FP32 &&
      cfg->precision != PINT_LEG_BF16X3) {
    set_error("pint_plan_create: precision must be PINT_FP64, PINT_LEG_FP32 or PINT_LEG_BF16X3 "
              "(got %d)",
              cfg->precision);
    return PINT_E_INVAL;
  }
  if (!(cfg->a > 0) || !(cfg->phibar >= 0) || cfg->max_batch < 1 || cfg->max_batch > 65535 ||
      !isfinite(cfg->omega) || !isfinite(cfg->g)) {
    set_error("pint_plan_create: need a > 0, phibar >= 0, finite omega/g, 1 <= max_batch <= 65535");
    return PINT_E_INVAL;
  }
  {
    int dev = 0, lds_max = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) !=
            hipSuccess) {
      set_error("pint_plan_create: cannot query the device");
      return PINT_E_HIP;
    }
    if (ring_lds_bytes(nlon, cfg->precision) > (size_t)lds_max) {
      set_error("pint_plan_create: nlon=%d needs %zu bytes of LDS per workgroup, device allows %d",
                nlon, ring_lds_bytes(nlon, cfg->precision), lds_max);
      return PINT_E_INVAL;
    }
    pint_status rs = ring_prepare(nlon);
    if (rs != PINT_OK) return rs;
  }
  pint_plan* pp = new pint_plan();
  Plan& p = pp->p;
  p.M = M;
  p.nlon = nlon;
  p.nlat = nlat;
  p.nlat2 = nlat / 2;
  p.ncoef = (M + 1) * (M + 2) / 2;
  p.a = cfg->a;
  p.omega = cfg->omega;
  p.g = cfg->g;
  p.phibar = cfg->phibar;
  p.max_batch = cfg->max_batch;
  p.prec = cfg->precision;

  // row space
  p.h_rowoff.assign(2 * (M + 1) + 1, 0);
  std::vector<int> rowinfo;
  for (int m = 0; m <= M; ++m) {
    for (int par = 0; par < 2; ++par) {
      p.h_rowoff[2 * m + par] = (int)rowinfo.size();
      for (int n = m + par; n <= M + 1; n += 2) rowinfo.push_back((m << 16) | n);
    }
  }
  p.h_rowoff[2 * (M + 1)] = (int)rowinfo.size();
  p.nrows = (int)rowinfo.size();
  std::vector<int> coefmn;
  for (int m = 0; m <= M; ++m)
    for (int n = m; n <= M; ++n) coefmn.push_back((m << 16) | n);

  size_t tot = 0;
  pint_status st = PINT_OK;
#define PLAN_TRY(x)       \
  do {                    \
    st = (x);             \
    if (st != PINT_OK) {  \
      free_plan(p);       \
      delete pp;          \
      return st;          \
    }                     \
  } while (0)
  PLAN_TRY(dalloc(&p.mu, nlat, &tot));
  PLAN_TRY(dalloc(&p.w, nlat, &tot));
  PLAN_TRY(dalloc(&p.c2, nlat, &tot));
  PLAN_TRY(dalloc(&p.ptab, (size_t)p.nrows * p.nlat2, &tot));
  PLAN_TRY(dalloc(&p.ptabT, (size_t)p.nrows * p.nlat2, &tot));
  PLAN_TRY(dalloc(&p.rowoff, p.h_rowoff.size(), &tot));
  PLAN_TRY(dalloc(&p.rowinfo, rowinfo.size(), &tot));
  PLAN_TRY(dalloc(&p.coefmn, coefmn.size(), &tot));
  PLAN_TRY(dalloc(&p.twid, nlon, &tot));
  if (p.prec != PINT_FP64) {
    PLAN_TRY(dalloc(&p.ptab32, (size_t)p.nrows * p.nlat2, &tot));
    PLAN_TRY(dalloc(&p.ptabT32, (size_t)p.nrows * p.nlat2, &tot));
    PLAN_TRY(dalloc(&p.twid32, nlon, &tot));
  }
  PLAN_TRY(dalloc(&p.cnco, p.ncoef, &tot));
  PLAN_TRY(build_tiles(p.h_rowoff, M, p.nlat2, true, kGemmTR, &p.syn_tiles, &tot));
  PLAN_TRY(build_tiles(p.h_rowoff, M, p.nlat2, false, kGemmTRAnal, &p.ana_tiles, &tot));
  PLAN_TRY(spec_tasks_build(p, &tot));
  const size_t B = p.max_batch;
  PLAN_TRY(dalloc(&p.S, (size_t)p.nrows * 12 * B, &tot));
  PLAN_TRY(dalloc(&p.F, (M + 1) * fourier_pitch<double>(nlat, 12 * B), &tot));
  PLAN_TRY(dalloc(&p.G, (M + 1) * fourier_pitch<double>(nlat, 8 * B), &tot));
  PLAN_TRY(dalloc(&p.Q, (size_t)p.nrows * 8 * B, &tot));
  const size_t sw = (size_t)p.ncoef * B * 3 * 2;
  PLAN_TRY(dalloc(&p.Ua, sw, &tot));
  PLAN_TRY(dalloc(&p.N1, sw, &tot));
  PLAN_TRY(dalloc(&p.side.S, (size_t)p.nrows * 12, &tot));
  PLAN_TRY(dalloc(&p.side.F, (M + 1) * fourier_pitch<double>(nlat, 12), &tot));
  PLAN_TRY(dalloc(&p.side.G, (M + 1) * fourier_pitch<double>(nlat, 8), &tot));
  PLAN_TRY(dalloc(&p.side.Q, (size_t)p.nrows * 8, &tot));
  PLAN_TRY(dalloc(&p.side.Ua, (size_t)p.ncoef * 3 * 2, &tot));
  PLAN_TRY(dalloc(&p.side.N1, (size_t)p.ncoef * 3 * 2, &tot));
  PLAN_TRY(dalloc(&p.red, (size_t)8 * B + 64, &tot));
  PLAN_TRY(dalloc(&p.diag, (size_t)6 * B * nlat, &tot));
  PLAN_TRY(dalloc(&p.sl_lat, (size_t)nlat + 4, &tot));
  if (hipHostMalloc((void**)&p.h_red, (8 * B + 64) * sizeof(double), 0) != hipSuccess) {
    free_plan(p);
    delete pp;
    set_error("hipHostMalloc failed");
    return PINT_E_NOMEM;
  }
  p.ws_bytes = tot;
  p.base_bytes = tot;
  // the sweep stream does not synchronise with the legacy null stream:
  // ordering against the caller's stream is by events only
  if (hipStreamCreateWithFlags(&p.side_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&p.capture_stream, hipStreamNonBlocking) != hipSuccess ||
      hipStreamCreateWithFlags(&p.relax_stream, hipStreamNonBlocking) != hipSuccess ||
      hipEventCreateWithFlags(&p.join_ev, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&p.relax_join_ev, hipEventDisableTiming) != hipSuccess) {
    free_plan(p);
    delete pp;
    set_error("hipStreamCreateWithFlags / hipEventCreateWithFlags failed");
    return PINT_E_HIP;
  }
  for (hipEvent_t& e : p.ph_ev) {
    if (hipEventCreate(&e) != hipSuccess) {
      free_plan(p);
      delete pp;
      set_error("hipEventCreate failed");
      return PINT_E_HIP;
    }
  }
  p.chunk_ev.assign(kMaxSweepChunks, nullptr);
  p.relax_ev.assign(kMaxSweepChunks, nullptr);
  p.relax_done_ev.assign(kMaxSweepChunks, nullptr);
  for (auto* v : {&p.relax_ev, &p.relax_done_ev})
    for (hipEvent_t& e : *v) {
      if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        free_plan(p);
        delete pp;
        set_error("hipEventCreateWithFlags failed");
        return PINT_E_HIP;
      }
    }
  for (hipEvent_t& e : p.chunk_ev) {
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      free_plan(p);
      delete pp;
      set_error("hipEventCreateWithFlags failed");
      return PINT_E_HIP;
    }
  }
  if (const char* env = getenv("PINT_GRAPHS")) p.use_graphs = atoi(env) != 0;
  if (const char* env = getenv("PINT_PIPELINE")) p.pipeline_relax = atoi(env) != 0;
  if (const char* env = getenv("PINT_GEMM_VARIANT")) {   // fixed launch shapes (tests)
    const int v = atoi(env) < 0 ? 0 : atoi(env);
    p.gemm_variant[0][0] = p.gemm_variant[1][0] = p.gemm_variant[0][1] = v > 1 ? 1 : v;
    p.gemm_variant[1][1] = v > 2 ? 2 : v;
    p.ring_variant[0] = p.ring_variant[1] = v > 1 ? 1 : v;
  }
  if (const char* env = getenv("PINT_SWEEP_CHUNKS")) {
    const int v = atoi(env);
    p.sweep_chunks = v < 1 ? 1 : (v > kMaxSweepChunks ? kMaxSweepChunks : v);
  }
  auto fail_hip = [&](hipError_t e, const char* what) {
    set_error("%s failed: %s", what, hipGetErrorString(e));
    free_plan(p);
    delete pp;
    return PINT_E_HIP;
  };
  hipError_t e;
  if ((e = hipMemcpyAsync(p.rowoff, p.h_rowoff.data(), p.h_rowoff.size() * sizeof(int),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail_hip(e, "hipMemcpyAsync(rowoff)");
  if ((e = hipMemcpyAsync(p.rowinfo, rowinfo.data(), rowinfo.size() * sizeof(int),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail_hip(e, "hipMemcpyAsync(rowinfo)");
  if ((e = hipMemcpyAsync(p.coefmn, coefmn.data(), coefmn.size() * sizeof(int),
                          hipMemcpyHostToDevice, s)) != hipSuccess)
    return fail_hip(e, "hipMemcpyAsync(coefmn)");
  hipLaunchKernelGGL(k_gauss, dim3((p.nlat2 + 63) / 64), dim3(64), 0, s, nlat, p.mu, p.w, p.c2);
  hipLaunchKernelGGL(k_ptab, dim3((p.nlat2 + 63) / 64, M + 1), dim3(64), 0, s, M, p.nlat2,
                     p.nrows, p.mu, p.c2, p.rowoff, p.ptab, p.ptabT);
  hipLaunchKernelGGL(k_twiddle, dim3((nlon + 255) / 256), dim3(256), 0, s, nlon, p.twid);
  hipLaunchKernelGGL(k_sl_lat, dim3((nlat + 4 + 63) / 64), dim3(64), 0, s, nlat, p.mu, p.sl_lat);
  if (p.prec != PINT_FP64) {
    const size_t nt = (size_t)p.nrows * p.nlat2;
    hipLaunchKernelGGL(k_to_float, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, p.ptab,
                       p.ptab32, nt);
    hipLaunchKernelGGL(k_to_float, dim3((unsigned)((nt + 255) / 256)), dim3(256), 0, s, p.ptabT,
                       p.ptabT32, nt);
    hipLaunchKernelGGL(k_to_float, dim3((unsigned)((2 * nlon + 255) / 256)), dim3(256), 0, s,
                       reinterpret_cast<const double*>(p.twid), reinterpret_cast<float*>(p.twid32),
                       (size_t)2 * nlon);
  }
  hipLaunchKernelGGL(k_cn_coef, dim3((p.ncoef + 255) / 256), dim3(256), 0, s, M, p.ncoef, p.a,
                     p.coefmn, p.cnco);
  if ((e = hipGetLastError()) != hipSuccess) return fail_hip(e, "table kernels");
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return fail_hip(e, "hipStreamSynchronize");
  // the device address of the library's static scratch on this device
  if ((st = noalloc_init_device()) != PINT_OK) {
    free_plan(p);
    delete pp;
    return st;
  }
  *out = pp;
  return PINT_OK;
#undef PLAN_TRY
}

// ---------------------------------------------------------------------------
// Kernel timing: events are taken from a pool that grows on demand (outside
// the kernels' critical path) and recycled by profile_read.
// ---------------------------------------------------------------------------
static hipEvent_t pool_event(Plan& p) {
  if (p.prof_used == p.ev_pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    p.ev_pool.push_back(e);
  }
  return p.ev_pool[p.prof_used++];
}

int prof_begin(Plan& p, int kind, int batch, hipStream_t s) {
  ProfRec r;
  r.kind = kind;
  r.batch = batch;
  r.a = pool_event(p);
  r.b = pool_event(p);
  if (!r.a || !r.b) return -1;
  if (hipEventRecord(r.a, s) != hipSuccess) return -1;
  p.prof.push_back(r);
  return (int)p.prof.size() - 1;
}

void prof_end(Plan& p, int rec, hipStream_t s) { (void)hipEventRecord(p.prof[rec].b, s); }

pint_status profile_read(Plan& p, pint_prof_entry* out, int cap, int* n, hipStream_t s) {
  PINT_HIP(hipStreamSynchronize(s));
  std::map<std::pair<int, int>, std::pair<long long, double>> acc;
  for (const ProfRec& r : p.prof) {
    float ms = 0.0f;
    PINT_HIP(hipEventElapsedTime(&ms, r.a, r.b));
    auto& e = acc[std::make_pair(r.kind, r.batch)];
    e.first += 1;
    e.second += ms;
  }
  int k = 0;
  for (auto& kv : acc) {
    if (k < cap && out) {
      out[k].kind = kv.first.first;
      out[k].batch = kv.first.second;
      out[k].launches = kv.second.first;
      out[k].total_ms = kv.second.second;
    }
    ++k;
  }
  if (n) *n = k < cap ? k : cap;
  p.prof.clear();
  p.prof_used = 0;
  return PINT_OK;
}

void destroy(pint_plan* pp) {
  if (!pp) return;
  (void)hipDeviceSynchronize();
  free_plan(pp->p);
  delete pp;
}

// ---------------------------------------------------------------------------
// Crank-Nicolson factors.  (I - alpha L) x = r with alpha = dt/4 (Sec. 2.3.1,
// eq. IMEX_implicit).  Eliminating Phi (x_Phi = r_Phi - alpha Phibar x_delta)
// leaves, per zonal wavenumber m, two tridiagonal chains
//   chain 0: (xi_m, delta_{m+1}, xi_{m+2}, ...), chain 1: (delta_m, xi_{m+1}, ...)
// because the implicit Coriolis term couples xi_n only to delta_{n+-1} (and
// to itself through i m psi_n), and delta_n only to xi_{n+-1}.  With
// s_k = -a^2/(k(k+1)) (s_0 = 0), eps_n = eps_n^m, W = 2 Omega:
//   (L u)_xi,n    = A_n delta_{n-1} + i B_n xi_n + C_n delta_{n+1}
//   (L u)_delta,n = n(n+1)/a^2 Phi_n - A_n xi_{n-1} + i B_n delta_n - C_n xi_{n+1}
//   A_n = -W eps_n + (W/a^2)(n-1) eps_n s_{n-1},   B_n = -(W/a^2) m s_n,
//   C_n = -W eps_{n+1} - (W/a^2)(n+2) eps_{n+1} s_{n+1}   (C_M = 0: truncation).
// One thread per (m, chain) runs the Thomas factorisation (no pivoting: the
// Hermitian part of I - alpha L is the identity in energy variables).
// ---------------------------------------------------------------------------
__global__ void k_cn_factor(int M, int ncoef, double a, double W, double phibar, double alpha,
                            int lg, double2* alph, double2* gam, double2* invpiv) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 2 * (M + 1)) return;
  const int m = t >> 1, chain = t & 1;
  const int K = M - m + 1;
  const size_t base = (size_t)chain * ncoef + coef_idx(M, m, m);
  double2 cpp = make_double2(0.0, 0.0);
  for (int i = 0; i < K; ++i) {
    const int n = m + i;
    const bool is_xi = ((i & 1) == 0) == (chain == 0);
    const CnCoef c = cn_coef(m, n, M, a, W, lg != 0);
    double2 l, d, u;
    if (is_xi) {
      l = make_double2(-alpha * c.A, 0.0);
      d = make_double2(1.0, -alpha * c.B);
      u = make_double2(-alpha * c.C, 0.0);
    } else {
      l = make_double2(alpha * c.A, 0.0);
      d = make_double2(1.0 + alpha * alpha * phibar * c.lap, -alpha * c.B);
      u = make_double2(alpha * c.C, 0.0);
    }
    const double2 lc = cmul(l, cpp);
    const double2 piv = make_double2(d.x - lc.x, d.y - lc.y);
    const double2 ip = cinv(piv);
    const double2 cp = cmul(u, ip);
    const double2 al = cmul(l, ip);
    alph[base + i] = make_double2(-al.x, -al.y);
    invpiv[base + i] = ip;
    gam[base + i] = make_double2(-cp.x, -cp.y);
    cpp = cp;
  }
}

// Factor set of (dt, terms) into the buffers of f (2 ncoef double2 each).
pint_status cn_factors_fill(const Plan& p, double dt, unsigned terms, const CnFactors& f,
                            hipStream_t s) {
  const unsigned key_terms = terms & (PINT_T_LG | PINT_T_LC);
  const double W = (key_terms & PINT_T_LC) ? 2.0 * p.omega : 0.0;
  const bool lg = (key_terms & PINT_T_LG) != 0;
  const int nt = 2 * (p.M + 1);
  hipLaunchKernelGGL(k_cn_factor, dim3((nt + 63) / 64), dim3(64), 0, s, p.M, p.ncoef, p.a, W,
                     lg ? p.phibar : 0.0, dt / 4.0, lg ? 1 : 0, f.alph, f.gam, f.invpiv);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status cn_factors(Plan& p, double dt, unsigned terms, hipStream_t s, const CnFactors** out) {
  const unsigned key_terms = terms & (PINT_T_LG | PINT_T_LC);
  auto key = std::make_pair(dt, key_terms);
  auto it = p.cn_cache.find(key);
  if (it != p.cn_cache.end()) {
    *out = &it->second;
    return PINT_OK;
  }
  CnFactors f;
  const size_t n = (size_t)2 * p.ncoef;
  p.n_allocs += 3;
  PINT_TRY(dalloc(&f.alph, n, &p.ws_bytes));
  PINT_TRY(dalloc(&f.gam, n, &p.ws_bytes));
  PINT_TRY(dalloc(&f.invpiv, n, &p.ws_bytes));
  PINT_TRY(cn_factors_fill(p, dt, terms, f, s));
  auto ins = p.cn_cache.emplace(key, f);
  *out = &ins.first->second;
  return PINT_OK;
}

size_t cn_factor_bytes(const Plan& p) { return (size_t)3 * 2 * p.ncoef * sizeof(double2); }

// Bytes a footprint adds to the plan's (and the coarse plan's) creation-time
// memory: pool slots at their needed sizes plus the factor sets.
size_t footprint_bytes(const Plan& p, const Plan* pc, const Footprint& fp) {
  size_t b = p.base_bytes;
  for (int i = 0; i < kSlotCount; ++i) b += fp.slot[i] * sizeof(double);
  b += fp.cn.size() * cn_factor_bytes(p);
  if (pc && pc != &p) b += fp.cn_coarse.size() * cn_factor_bytes(*pc);
  else b += fp.cn_coarse.size() * cn_factor_bytes(p);
  return b;
}

pint_status reserve(Plan& p, Plan* pc, const Footprint& fp, hipStream_t s) {
  if (fp.host_doubles > p.h_incr_n) {
    if (p.h_incr) (void)hipHostFree(p.h_incr);
    p.h_incr = nullptr;
    p.h_incr_n = 0;
    ++p.n_allocs;
    if (hipHostMalloc((void**)&p.h_incr, fp.host_doubles * sizeof(double), 0) != hipSuccess) {
      p.h_incr = nullptr;
      set_error("hipHostMalloc(%zu bytes) failed", fp.host_doubles * sizeof(double));
      return PINT_E_NOMEM;
    }
    p.h_incr_n = fp.host_doubles;
  }
  for (int i = 0; i < kSlotCount; ++i)
    if (fp.slot[i]) {
      DevBuf b(p, i);
      PINT_TRY(b.alloc(fp.slot[i]));
    }
  const CnFactors* f = nullptr;
  for (const auto& k : fp.cn) PINT_TRY(cn_factors(p, k.first, k.second, s, &f));
  Plan& c = pc ? *pc : p;
  for (const auto& k : fp.cn_coarse) PINT_TRY(cn_factors(c, k.first, k.second, s, &f));
  return PINT_OK;
}

}  // namespace pint
