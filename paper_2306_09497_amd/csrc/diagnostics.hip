// Diagnostics of Sec. 5 and Sec. 5.1 on the device, over states in the public
// layout [B][3][ncoef][2]:
//   * the kinetic-energy spectrum of a triangular truncation,
//       E(n) = a^2 / (4 n (n+1)) sum_{m=-n..n} (|xi_{m,n}|^2 + |delta_{m,n}|^2),
//     the m < 0 partners being the conjugates of a real field's m > 0
//     coefficients (so those terms count twice);
//   * the spectral max-norm errors E_{psi,R} (eq. error_definition) of
//     psi = Phi', xi, delta for every resolution R = 0..M at once:
//     the largest modulus of the difference over m <= n <= R over the largest
//     reference modulus there (Phi' = Phi - Phibar; a zero reference norm
//     gives 0 for a zero difference, +inf otherwise);
//   * the pair spectra (psi - psi_ref, psi_ref) whose grid-point sums of
//     squares give the physical-space L2 errors (unnumbered equation after
//     error_definition) on the Gauss grid: synthesised by the scalar
//     Legendre GEMM and summed per ring by the scalar ring kernel.
// Small, HBM-light kernels: one pass over the coefficients each.
#include "pint_internal.h"

namespace pint {
namespace {

__device__ inline double2 load_c(const double* p, size_t i) {
  return *reinterpret_cast<const double2*>(p + 2 * i);
}

// 64 n of one state per workgroup, four waves splitting m by m mod 4:
// threads of consecutive n read consecutive coefficients of each m; each
// wave sums its m in increasing order, then the four partial sums are added
// in wave order.
constexpr int kKeWaves = 4;
__global__ __launch_bounds__(64 * kKeWaves) void k_ke_spectrum(const double* __restrict__ u,
                                                               double* __restrict__ e, int M,
                                                               int ncoef, double a2) {
  __shared__ double part[kKeWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int n = blockIdx.x * 64 + lane, b = blockIdx.y;
  const double* xi = u + ((size_t)b * 3 + 1) * ncoef * 2;
  const double* de = xi + (size_t)ncoef * 2;
  double s = 0.0;
  if (n <= M) {
    for (int m = w; m <= n; m += kKeWaves) {
      const int k = coef_idx(M, m, n);
      const double2 x = load_c(xi, k), d = load_c(de, k);
      const double v = (x.x * x.x + x.y * x.y) + (d.x * d.x + d.y * d.y);
      s += m == 0 ? v : 2.0 * v;
    }
  }
  part[w][lane] = s;
  __syncthreads();
  if (w == 0 && n <= M) {
    double t = part[0][lane];
    for (int q = 1; q < kKeWaves; ++q) t += part[q][lane];
    e[(size_t)b * (M + 1) + n] = n == 0 ? 0.0 : 0.25 * a2 / (n * (n + 1.0)) * t;
  }
}

constexpr int kErrThreads = 256;
constexpr int kErrMaxN = 512;          // M <= 511 (nlon <= 1024)

// One workgroup per (state, field): per n the largest moduli over m <= n of
// the difference and of the reference, then an inclusive running maximum
// over n gives every R at once.
__global__ __launch_bounds__(kErrThreads) void k_spectral_errors(
    const double* __restrict__ u, const double* __restrict__ ref, double* __restrict__ out, int M,
    int ncoef, double phibar) {
  __shared__ double cd[kErrMaxN], cr[kErrMaxN];
  const int bf = blockIdx.x, f = bf % 3;
  const double* x = u + (size_t)bf * ncoef * 2;
  const double* y = ref + (size_t)bf * ncoef * 2;
  for (int n = threadIdx.x; n <= M; n += kErrThreads) {
    double md = 0.0, mr = 0.0;
    for (int m = 0; m <= n; ++m) {
      const int k = coef_idx(M, m, n);
      double2 xv = load_c(x, k), yv = load_c(y, k);
      if (f == 0 && k == 0) {          // Phi' = Phi - Phibar
        xv.x -= phibar;
        yv.x -= phibar;
      }
      const double dx = xv.x - yv.x, dy = xv.y - yv.y;
      md = fmax(md, sqrt(dx * dx + dy * dy));
      mr = fmax(mr, sqrt(yv.x * yv.x + yv.y * yv.y));
    }
    cd[n] = md;
    cr[n] = mr;
  }
  __syncthreads();
  for (int off = 1; off <= M; off <<= 1) {
    double vd[kErrMaxN / kErrThreads], vr[kErrMaxN / kErrThreads];
#pragma unroll
    for (int i = 0; i < kErrMaxN / kErrThreads; ++i) {
      const int n = threadIdx.x + i * kErrThreads;
      vd[i] = (n <= M && n >= off) ? fmax(cd[n], cd[n - off]) : 0.0;
      vr[i] = (n <= M && n >= off) ? fmax(cr[n], cr[n - off]) : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kErrMaxN / kErrThreads; ++i) {
      const int n = threadIdx.x + i * kErrThreads;
      if (n <= M && n >= off) {
        cd[n] = vd[i];
        cr[n] = vr[i];
      }
    }
    __syncthreads();
  }
  for (int R = threadIdx.x; R <= M; R += kErrThreads) {
    const double num = cd[R], den = cr[R];
    out[(size_t)bf * (M + 1) + R] = den > 0.0 ? num / den : (num == 0.0 ? 0.0 : INFINITY);
  }
}

// Synthesis input for the L2 errors: spectrum q = 6 b + 2 f + k of the nb
// states, k = 0 the difference psi - psi_ref, k = 1 the reference, in the
// row space of the Legendre GEMM (rows with n = M + 1 are zero).
__global__ void k_l2_pairs(const double* __restrict__ u, const double* __restrict__ ref,
                           double* __restrict__ S, const int* __restrict__ rowinfo, int nrows,
                           int M, int ncoef, int nb, double phibar) {
  const int ns = 6 * nb;
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)nrows * ns) return;
  const int q = (int)(t % ns), row = (int)(t / ns);
  const int b = q / 6, f = (q >> 1) % 3, k = q & 1;
  const int mn = rowinfo[row];
  const int m = mn >> 16, n = mn & 0xffff;
  double2 v = make_double2(0.0, 0.0);
  if (n <= M) {
    const int c = coef_idx(M, m, n);
    double2 xv = load_c(u, ((size_t)b * 3 + f) * ncoef + c);
    double2 yv = load_c(ref, ((size_t)b * 3 + f) * ncoef + c);
    if (f == 0 && c == 0) {
      xv.x -= phibar;
      yv.x -= phibar;
    }
    v = k == 0 ? make_double2(xv.x - yv.x, xv.y - yv.y) : yv;
  }
  *reinterpret_cast<double2*>(S + 2 * t) = v;
}

}  // namespace

pint_status ke_spectrum(Plan& p, const double* u, double* e, int B, hipStream_t s) {
  if (B == 0) return PINT_OK;
  hipLaunchKernelGGL(k_ke_spectrum, dim3((p.M + 64) / 64, B), dim3(64 * kKeWaves), 0, s, u, e,
                     p.M, p.ncoef, p.a * p.a);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status spectral_errors(Plan& p, const double* u, const double* ref, double* e, int B,
                            hipStream_t s) {
  if (B == 0) return PINT_OK;
  if (p.M >= kErrMaxN) {
    set_error("spectral errors support M < %d (got %d)", kErrMaxN, p.M);
    return PINT_E_INVAL;
  }
  hipLaunchKernelGGL(k_spectral_errors, dim3(3 * B), dim3(kErrThreads), 0, s, u, ref, e, p.M,
                     p.ncoef, p.phibar);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status grid_l2_errors(Plan& p, const double* u, const double* ref, double* out_host, int B,
                           hipStream_t s) {
  std::vector<double> part;
  for (int b0 = 0; b0 < B; b0 += p.max_batch) {
    const int nb = (B - b0) < p.max_batch ? (B - b0) : p.max_batch;
    const size_t sd = (size_t)3 * p.ncoef * 2 * b0;
    const size_t total = (size_t)p.nrows * 6 * nb;
    hipLaunchKernelGGL(k_l2_pairs, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, u + sd,
                       ref + sd, p.S, p.rowinfo, p.nrows, p.M, p.ncoef, nb, p.phibar);
    PINT_HIP(hipGetLastError());
    PINT_TRY(legendre_synth(p, 6 * nb, 1, PINT_FP64, s));
    PINT_TRY(ring_sumsq(p, 6 * nb, p.diag, s));
    // partial sums [pair = 3 b + f][latitude][difference, reference]
    part.resize((size_t)3 * nb * p.nlat * 2);
    PINT_HIP(hipMemcpyAsync(part.data(), p.diag, part.size() * sizeof(double),
                            hipMemcpyDeviceToHost, s));
    PINT_HIP(hipStreamSynchronize(s));
    for (int q = 0; q < 3 * nb; ++q) {
      double num = 0.0, den = 0.0;
      for (int j = 0; j < p.nlat; ++j) {
        num += part[((size_t)q * p.nlat + j) * 2];
        den += part[((size_t)q * p.nlat + j) * 2 + 1];
      }
      out_host[(size_t)b0 * 3 + q] =
          den > 0.0 ? std::sqrt(num / den) : (num == 0.0 ? 0.0 : INFINITY);
    }
  }
  return PINT_OK;
}

}  // namespace pint
