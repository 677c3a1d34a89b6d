// Legendre transforms as ragged batched FP64 GEMMs on the CDNA matrix cores
// (v_mfma_f64_16x16x4_f64).  Sec. 2.2: per zonal wavenumber m the Legendre
// transform is a dense contraction between the table Pbar_n^m(mu_j) and all
// columns (fields x batch x re/im) at once.  The equatorial symmetry
// Pbar_n^m(-mu) = (-1)^(n-m) Pbar_n^m(mu) splits each m into an even and an odd
// problem p = 2m + par over the northern latitudes only (half the flops):
//
//   synthesis: F[p][jn][c] = sum_k T[row(p,k)][jn] * S[row(p,k)][c]
//              (even/odd partial sums E, O; the ring kernel forms E +- O)
//   analysis:  Q[row(p,r)][c] = sum_jn T[row(p,r)][jn] *
//                               (G[m][jn][c] + (-1)^par G[m][nlat-1-jn][c])
//
// T is the row-space table [nrows][nlat2].  Reduction order over k is fixed
// and independent of the column tiling and tile width, so results are
// batch-invariant.
#include "pint_internal.h"

namespace pint {

typedef double v4d __attribute__((ext_vector_type(4)));

// Tile: TR = 64 rows x TC columns (TC = 64 for batched launches, 16 for the
// latency-bound single-state launches of the serial coarse sweep), k-slabs of
// TK = 16 double-buffered in LDS: the next slab is fetched into registers
// while the matrix cores work on the current one, one barrier per slab.
template <bool kSynth, int TR, int TC>
__global__ __launch_bounds__(256) void k_legendre(const double* __restrict__ T,
                                                  const int* __restrict__ rowoff,
                                                  const int* __restrict__ tiles,
                                                  const double* __restrict__ Bsrc,
                                                  double* __restrict__ C, int nlat, int nlat2,
                                                  int ncol) {
  constexpr int TK = kGemmTK;
  constexpr int LDA = TR + 2, LDB = TC + 2;
  constexpr int NA = TK * TR / 256;                  // A elements per thread per slab
  constexpr int NB = TK * TC / 256;                  // B elements per thread per slab
  constexpr int WC = TC == 64 ? 2 : 1;               // waves across columns
  constexpr int WR = 4 / WC;                         // waves across rows
  constexpr int BI = TR / WR / 16, BJ = TC / WC / 16;  // MFMA blocks per wave
  static_assert(BI >= 1 && BJ >= 1 && NA >= 1 && NB >= 1, "tile shape");
  __shared__ double As[2][TK * LDA];
  __shared__ double Bs[2][TK * LDB];

  // logical block = row tile * ncoltiles + column tile (column tiles of one
  // table tile adjacent), XCD-remapped so that they share an L2; the tile
  // list is ordered so that each XCD's range holds an equal share of work
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int nct = (ncol + TC - 1) / TC;
  const int rt = lb / nct;
  const int p = tiles[2 * rt];
  const int row0 = tiles[2 * rt + 1];
  const int m = p >> 1, par = p & 1;
  const int roff = rowoff[p];
  const int cnt = rowoff[p + 1] - roff;
  const int col0 = (lb - rt * nct) * TC;
  const int R = kSynth ? nlat2 : cnt;
  const int K = kSynth ? cnt : nlat2;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave / WC) * (TR / WR), wc = (wave % WC) * (TC / WC);
  const int li = lane & 15, lk = lane >> 4;
  const double sgn = par ? -1.0 : 1.0;
  const size_t gbase = (size_t)m * nlat;

  v4d acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

  double ra[NA], rb[NB];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * 256;
      double v = 0.0;
      if (kSynth) {
        const int kk = e / TR, rr = e % TR;
        const int k = k0 + kk, r = row0 + rr;
        if (k < K && r < R) v = T[(size_t)(roff + k) * nlat2 + r];
      } else {
        const int rr = e / TK, kk = e % TK;
        const int k = k0 + kk, r = row0 + rr;
        if (k < K && r < R) v = T[(size_t)(roff + r) * nlat2 + k];
      }
      ra[q] = v;
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * 256;
      const int kk = e / TC, cc = e % TC;
      const int k = k0 + kk, c = col0 + cc;
      double v = 0.0;
      if (k < K && c < ncol) {
        if (kSynth)
          v = Bsrc[(size_t)(roff + k) * ncol + c];
        else
          v = Bsrc[(gbase + k) * ncol + c] + sgn * Bsrc[(gbase + (nlat - 1 - k)) * ncol + c];
      }
      rb[q] = v;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = tid + q * 256;
      if (kSynth)
        As[buf][(e / TR) * LDA + (e % TR)] = ra[q];
      else
        As[buf][(e % TK) * LDA + (e / TK)] = ra[q];
    }
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const int e = tid + q * 256;
      Bs[buf][(e / TC) * LDB + (e % TC)] = rb[q];
    }
  };

  const int nslab = (K + TK - 1) / TK;
  if (nslab > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  for (int sl = 0; sl < nslab; ++sl) {
    const int cur = sl & 1;
    if (sl + 1 < nslab) fetch((sl + 1) * TK);
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      double a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = As[cur][(ks + lk) * LDA + wr + 16 * i + li];
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = Bs[cur][(ks + lk) * LDB + wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (sl + 1 < nslab) stash(cur ^ 1);
    __syncthreads();
  }
  // ---- store: on gfx950 lane l, register i of a 16x16 f64 block holds
  //      D[l/16 + 4 i][l % 16] ----
#pragma unroll
  for (int bi = 0; bi < BI; ++bi) {
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      const int c = col0 + wc + bj * 16 + li;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = row0 + wr + bi * 16 + lk + 4 * i;
        if (r < R && c < ncol) {
          const size_t orow = kSynth ? (size_t)p * nlat2 + r : (size_t)(roff + r);
          C[orow * ncol + c] = acc[bi][bj][i];
        }
      }
    }
  }
}

// Synthesis rows are the nlat/2 latitudes (64-row tiles); analysis rows are
// the ragged n-range of one (m, parity) (32-row tiles waste less of it).
// Single-state launches use 64 x 16 tiles; batched ones 64 x 64 (synthesis)
// or 32 x 64 (analysis).  Every shape reduces over k in the same order.
template <bool kSynth>
static pint_status launch_legendre(Plan& p, const GemmTiles& narrow, const GemmTiles& wide,
                                   const double* Bsrc, double* C, int ncol, hipStream_t s) {
  constexpr int TRW = kSynth ? kGemmTR : kGemmTRAnal;
  if (ncol <= 32) {
    dim3 grid(((ncol + 15) / 16) * narrow.count);
    hipLaunchKernelGGL((k_legendre<kSynth, kGemmTR, 16>), grid, dim3(256), 0, s, p.ptab,
                       p.rowoff, narrow.dev, Bsrc, C, p.nlat, p.nlat2, ncol);
  } else {
    dim3 grid(((ncol + 63) / 64) * wide.count);
    hipLaunchKernelGGL((k_legendre<kSynth, TRW, 64>), grid, dim3(256), 0, s, p.ptab, p.rowoff,
                       wide.dev, Bsrc, C, p.nlat, p.nlat2, ncol);
  }
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status legendre_synth(Plan& p, int B, int nf, hipStream_t s) {
  ProfScope ps(p, PK_SYNTH, nf == kSynFields ? B : -B, s);
  return launch_legendre<true>(p, p.syn_tiles, p.syn_tiles, p.S, p.F, 2 * nf * B, s);
}

pint_status legendre_anal(Plan& p, int B, int nf, hipStream_t s) {
  ProfScope ps(p, PK_ANAL, nf == kAnaFields ? B : -B, s);
  return launch_legendre<false>(p, p.ana_tiles64, p.ana_tiles, p.G, p.Q, 2 * nf * B, s);
}

}  // namespace pint
