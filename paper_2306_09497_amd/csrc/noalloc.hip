// pint_step_noalloc: the IMEX propagator of pint_step with every buffer
// beyond the caller's states and the plan's tables in one static device
// array (`scratch`), for callers that cannot allocate device memory.
//
// Layout of the scratch of one call (byte offsets, 256-byte aligned):
//   [0, cn)        Crank-Nicolson factors of the call's stepper: alph, gam,
//                  invpiv, 2 ncoef double2 each (made by a kernel per call)
//   [cn, ...)      the transform workspace of one chunk of b states: S, F,
//                  G, Q, Ua, N1, sized as the plan's own for b states
// b is the largest chunk (at most the plan's max_batch) that fits; the
// states are propagated chunk after chunk.  Every call on a device shares
// that device's array and overwrites what it needs before reading it
// (nothing has to start at zero); calls that overlap in time on one device
// race on it.
#include <mutex>

#include "pint_internal.h"

namespace pint {

constexpr size_t kScratchBytes = (size_t)64 << 20;   // 64 MiB per device
constexpr int kMaxDevices = 64;

static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

// Device address of `scratch` per device (the host-side name is not one).
static double* g_scratch[kMaxDevices] = {};
static std::mutex g_scratch_mu;

pint_status noalloc_init_device() {
  int dev = 0;
  PINT_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index %d beyond the %d the library supports", dev, kMaxDevices);
    return PINT_E_INVAL;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return PINT_OK;
  void* ptr = nullptr;
  PINT_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
  if (!ptr) {
    set_error("hipGetSymbolAddress(scratch) returned a null address");
    return PINT_E_HIP;
  }
  g_scratch[dev] = static_cast<double*>(ptr);
  return PINT_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of the transform workspace of b states (the plan's buffers at b).
static size_t work_bytes(const Plan& p, int b) {
  const size_t d = sizeof(double);
  return align256((size_t)p.nrows * 12 * b * d) +
         align256((size_t)(p.M + 1) * fourier_pitch<double>(p.nlat, 12 * b) * d) +
         align256((size_t)(p.M + 1) * fourier_pitch<double>(p.nlat, 8 * b) * d) +
         align256((size_t)p.nrows * 8 * b * d) + 2 * align256((size_t)p.ncoef * b * 3 * 2 * d);
}

// Points the plan's workspace at the scratch while in scope (kernels capture
// the pointers current at their enqueue).
struct ScratchWork {
  Plan& p;
  double *S, *F, *G, *Q, *Ua, *N1;
  ScratchWork(Plan& pl, char* base, int b) : p(pl) {
    S = p.S, F = p.F, G = p.G, Q = p.Q, Ua = p.Ua, N1 = p.N1;
    const size_t d = sizeof(double);
    auto take = [&](size_t bytes) {
      double* r = reinterpret_cast<double*>(base);
      base += align256(bytes);
      return r;
    };
    p.S = take((size_t)p.nrows * 12 * b * d);
    p.F = take((size_t)(p.M + 1) * fourier_pitch<double>(p.nlat, 12 * b) * d);
    p.G = take((size_t)(p.M + 1) * fourier_pitch<double>(p.nlat, 8 * b) * d);
    p.Q = take((size_t)p.nrows * 8 * b * d);
    p.Ua = take((size_t)p.ncoef * b * 3 * 2 * d);
    p.N1 = take((size_t)p.ncoef * b * 3 * 2 * d);
  }
  ~ScratchWork() { p.S = S, p.F = F, p.G = G, p.Q = Q, p.Ua = Ua, p.N1 = N1; }
};

}  // namespace pint

using namespace pint;

extern "C" pint_status pint_step_noalloc(pint_plan* plan, const pint_stepper* st,
                                         const double* u_in, double* u_out, int B, int nsteps,
                                         void* stream) {
  if (!plan) {
    set_error("null plan");
    return PINT_E_INVAL;
  }
  Plan& p = plan->p;
  PINT_TRY(check_stepper(p, st));
  if (B < 0 || nsteps < 0 || (B > 0 && (!u_in || !u_out))) {
    set_error("need B >= 0, nsteps >= 0 and non-null state arrays");
    return PINT_E_INVAL;
  }
  hipStream_t s = (hipStream_t)stream;
  const size_t sd = (size_t)3 * p.ncoef * 2;
  if (B == 0) return PINT_OK;
  if (nsteps == 0) {
    if (u_in != u_out)
      PINT_HIP(hipMemcpyAsync(u_out, u_in, (size_t)B * sd * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    return PINT_OK;
  }
  int dev = 0;
  PINT_HIP(hipGetDevice(&dev));
  double* base = (dev >= 0 && dev < kMaxDevices) ? g_scratch[dev] : nullptr;
  if (!base) {
    set_error("no scratch set up on device %d: create a plan on it first", dev);
    return PINT_E_INVAL;
  }
  const size_t cn = align256((size_t)2 * p.ncoef * sizeof(double2));
  const size_t room = kScratchBytes - 3 * cn;
  int b = B < p.max_batch ? B : p.max_batch;
  while (b > 0 && work_bytes(p, b) > room) --b;
  if (b == 0) {
    set_error("one state at M = %d needs %zu bytes of scratch, the maximum is %zu", p.M,
              3 * cn + work_bytes(p, 1), kScratchBytes);
    return PINT_E_INVAL;
  }
  char* bytes = reinterpret_cast<char*>(base);
  CnFactors f;
  f.alph = reinterpret_cast<double2*>(bytes);
  f.gam = reinterpret_cast<double2*>(bytes + cn);
  f.invpiv = reinterpret_cast<double2*>(bytes + 2 * cn);
  PINT_TRY(cn_factors_fill(p, st->dt, st->terms, f, s));
  ScratchWork sw(p, bytes + 3 * cn, b);
  for (int b0 = 0; b0 < B; b0 += b) {
    const int nb = (B - b0) < b ? (B - b0) : b;
    PINT_TRY(imex_steps(p, *st, u_in + b0 * sd, u_out + b0 * sd, nb, nsteps, s, nullptr, nullptr,
                        false, false, &f));
  }
  return PINT_OK;
}
