// Legendre transforms as ragged batched FP64 GEMMs on the CDNA matrix cores
// (v_mfma_f64_16x16x4_f64).  Sec. 2.2: per zonal wavenumber m the Legendre
// transform is a dense contraction between the table Pbar_n^m(mu_j) and all
// columns (fields x batch x re/im) at once.  The equatorial symmetry
// Pbar_n^m(-mu) = (-1)^(n-m) Pbar_n^m(mu) splits each m into an even and an odd
// problem p = 2m + par over the northern latitudes only (half the flops):
//
//   synthesis: E/O[jn][c] = sum_k T[row(p,k)][jn] * S[row(p,k)][c], p = 2m, 2m+1,
//              F[m][jn][c] = E + O,  F[m][nlat-1-jn][c] = E - O
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
// TK = 16 double-buffered in LDS: the next slab is fetched into registers while the
// matrix cores work on the current one, one barrier per slab.  The matrix
// cores consume k in steps of 4 in increasing order whatever TK and TC are,
// so every launch shape gives bitwise the same sums.
// A synthesis tile covers both parities of its m (two accumulators) and its
// epilogue writes the latitude pairs: F[m][j] = E + O (north, j < nlat/2),
// F[m][nlat-1-j] = E - O (south).
template <bool kSynth, int TR, int TC, int TK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_legendre(
                                                  const double* __restrict__ T,
                                                  const int* __restrict__ rowoff,
                                                  const int* __restrict__ tiles,
                                                  const double* __restrict__ Bsrc,
                                                  double* __restrict__ C, int nlat, int nlat2,
                                                  int ncol) {
  constexpr int LDA = TR + 2, LDB = TC + 2;
  constexpr int NA = TK * TR / 256;                  // A elements per thread per slab
  constexpr int NB = TK * TC / 256;                  // B elements per thread per slab
  constexpr int WC = TC == 64 ? 2 : 1;               // waves across columns
  constexpr int WR = 4 / WC;                         // waves across rows
  constexpr int BI = TR / WR / 16, BJ = TC / WC / 16;  // MFMA blocks per wave
  constexpr int NPAR = kSynth ? 2 : 1;               // parities per tile
  static_assert(BI >= 1 && BJ >= 1 && NA >= 1 && NB >= 1, "tile shape");
  __shared__ double As[2][TK * LDA];
  __shared__ double Bs[2][TK * LDB];

  // logical block = row tile * ncoltiles + column tile (column tiles of one
  // table tile adjacent), XCD-remapped so that they share an L2; the tile
  // list is ordered so that each XCD's range holds an equal share of work
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int nct = (ncol + TC - 1) / TC;
  const int rt = lb / nct;
  const int p0 = tiles[2 * rt];
  const int row0 = tiles[2 * rt + 1];
  const int m = p0 >> 1;
  const int col0 = (lb - rt * nct) * TC;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave / WC) * (TR / WR), wc = (wave % WC) * (TC / WC);
  const int li = lane & 15, lk = lane >> 4;
  const size_t gbase = (size_t)m * nlat;

  v4d acc[NPAR][BI][BJ];
#pragma unroll
  for (int q = 0; q < NPAR; ++q)
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j) acc[q][i][j] = (v4d){0.0, 0.0, 0.0, 0.0};

  // slabs of the tile: parity 0 then (synthesis) parity 1, one pipeline
  const int roff0 = rowoff[kSynth ? 2 * m : p0];
  const int cnt0 = rowoff[(kSynth ? 2 * m : p0) + 1] - roff0;
  const int K0 = kSynth ? cnt0 : nlat2;
  const int ns0 = (K0 + TK - 1) / TK;
  int roff1 = 0, K1 = 0, ns1 = 0;
  if constexpr (kSynth) {
    roff1 = rowoff[2 * m + 1];
    K1 = rowoff[2 * m + 2] - roff1;
    ns1 = (K1 + TK - 1) / TK;
  }
  const int R = kSynth ? nlat2 : cnt0;
  const double sgn = (p0 & 1) ? -1.0 : 1.0;          // analysis: parity of the problem
  double ra[NA], rb[NB];
  auto fetch = [&](int sl) {
    const bool second = kSynth && sl >= ns0;
    const int roff = second ? roff1 : roff0;
    const int K = second ? K1 : K0;
    const int k0 = (second ? sl - ns0 : sl) * TK;
#pragma unroll
    for (int e4 = 0; e4 < NA; ++e4) {
      const int e = tid + e4 * 256;
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
      ra[e4] = v;
    }
#pragma unroll
    for (int e4 = 0; e4 < NB; ++e4) {
      const int e = tid + e4 * 256;
      const int kk = e / TC, cc = e % TC;
      const int k = k0 + kk, c = col0 + cc;
      double v = 0.0;
      if (k < K && c < ncol) {
        if (kSynth)
          v = Bsrc[(size_t)(roff + k) * ncol + c];
        else
          v = Bsrc[(gbase + k) * ncol + c] + sgn * Bsrc[(gbase + (nlat - 1 - k)) * ncol + c];
      }
      rb[e4] = v;
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e4 = 0; e4 < NA; ++e4) {
      const int e = tid + e4 * 256;
      if (kSynth)
        As[buf][(e / TR) * LDA + (e % TR)] = ra[e4];
      else
        As[buf][(e % TK) * LDA + (e / TK)] = ra[e4];
    }
#pragma unroll
    for (int e4 = 0; e4 < NB; ++e4) {
      const int e = tid + e4 * 256;
      Bs[buf][(e / TC) * LDB + (e % TC)] = rb[e4];
    }
  };
  auto mma = [&](int cur, v4d (&ac)[BI][BJ]) {
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
          ac[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], ac[i][j], 0, 0, 0);
    }
  };

  const int nslab = ns0 + ns1;
  if (nslab > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  // parity 0 slabs (the last one prefetches parity 1's first), then parity 1
#pragma unroll
  for (int q = 0; q < NPAR; ++q) {
    for (int sl = q ? ns0 : 0; sl < (q ? nslab : ns0); ++sl) {
      const int cur = sl & 1;
      if (sl + 1 < nslab) fetch(sl + 1);
      mma(cur, acc[q]);
      if (sl + 1 < nslab) stash(cur ^ 1);
      __syncthreads();
    }
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
        if constexpr (kSynth) {
          if (r < nlat2 && c < ncol) {
            const double e = acc[0][bi][bj][i], o = acc[NPAR - 1][bi][bj][i];
            C[(gbase + r) * ncol + c] = e + o;
            C[(gbase + (nlat - 1 - r)) * ncol + c] = e - o;
          }
        } else {
          const int cnt = rowoff[p0 + 1] - rowoff[p0];
          if (r < cnt && c < ncol) C[(size_t)(rowoff[p0] + r) * ncol + c] = acc[0][bi][bj][i];
        }
      }
    }
  }
}

// Synthesis rows are the nlat/2 latitudes; analysis rows are the ragged
// n-range of one (m, parity).  Single-state launches use 64 x 16 tiles,
// batched ones 64 x 64 tiles.  Every shape reduces over k in the same order.
template <bool kSynth>
static pint_status launch_legendre(Plan& p, const GemmTiles& narrow, const GemmTiles& wide,
                                   const double* Bsrc, double* C, int ncol, hipStream_t s) {
  constexpr int TRW = kSynth ? kGemmTR : kGemmTRAnal;
  if (ncol <= 32) {
    dim3 grid(((ncol + 15) / 16) * narrow.count);
    hipLaunchKernelGGL((k_legendre<kSynth, kGemmTR, 16, kGemmTK>), grid, dim3(256), 0, s,
                       p.ptab, p.rowoff, narrow.dev, Bsrc, C, p.nlat, p.nlat2, ncol);
  } else {
    dim3 grid(((ncol + 63) / 64) * wide.count);
    hipLaunchKernelGGL((k_legendre<kSynth, TRW, 64, kGemmTK>), grid, dim3(256), 0, s, p.ptab,
                       p.rowoff, wide.dev, Bsrc, C, p.nlat, p.nlat2, ncol);
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
