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
// A tile always covers both parities of its m, so the E/O combination costs
// no extra loads.  T is the row-space table [nrows][nlat2] (synthesis) or its
// transpose [nlat2][nrows] (analysis: rows contiguous).  Reduction order over
// k is fixed and independent of the tiling, so results are batch-invariant.
#include "pint_internal.h"

namespace pint {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));

// One 16x16x4 matrix-core product per element type.  Operand layouts are the
// same for FP64 and FP32 (lane l holds A[l%16][l/16] and B[l/16][l%16]); the
// result layouts differ (measured on gfx950 with in-bounds probes): register
// i of lane l holds D[l/16 + 4i][l%16] for FP64, D[4(l/16) + i][l%16] for FP32.
template <typename T>
struct Mma;
template <>
struct Mma<double> {
  typedef v4d acc_t;
  __device__ static inline acc_t zero() { return (v4d){0.0, 0.0, 0.0, 0.0}; }
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int i) { return lk + 4 * i; }
};
template <>
struct Mma<float> {
  typedef v4f acc_t;
  __device__ static inline acc_t zero() { return (v4f){0.0f, 0.0f, 0.0f, 0.0f}; }
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int row(int lk, int i) { return 4 * lk + i; }
};

// Synthesis tile: TR = 64 latitudes x TC columns (TC = 64 for batched
// launches, 16 for the latency-bound single-state launches of the serial
// coarse sweep), k-slabs of TK = 16 double-buffered in LDS: the next slab is
// fetched into registers while the matrix cores work on the current one, one
// barrier per slab.  A tile runs both parities of its m through one slab
// pipeline into two accumulators, and its epilogue writes the latitude pairs
// F[m][j] = E + O (north, j < nlat/2) and F[m][nlat-1-j] = E - O (south).
// The matrix cores consume k in steps of 4 in increasing order whatever TC
// is, so every launch shape gives bitwise the same sums.
template <typename E, int TR, int TC, int TK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_legendre_synth(
    const E* __restrict__ T, const int* __restrict__ rowoff, const int* __restrict__ tiles,
    const E* __restrict__ S, E* __restrict__ F, int nlat, int nlat2, int ncol) {
  using MM = Mma<E>;
  constexpr int LDA = TR + 2, LDB = TC + 2;
  constexpr int NA = TK * TR / 256;                  // A elements per thread per slab
  constexpr int NB = TK * TC / 256;                  // B elements per thread per slab
  constexpr int WC = TC >= 64 ? 2 : 1;               // waves across columns
  constexpr int WR = 4 / WC;                         // waves across rows
  constexpr int BI = TR / WR / 16, BJ = TC / WC / 16;  // MFMA blocks per wave
  static_assert(BI >= 1 && BJ >= 1 && NA >= 1 && NB >= 1, "tile shape");
  __shared__ E As[2][TK * LDA];
  __shared__ E Bs[2][TK * LDB];

  // logical block = row tile * ncoltiles + column tile (column tiles of one
  // table tile adjacent), XCD-remapped so that they share an L2; the tile
  // list is ordered so that each XCD's range holds an equal share of work
  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int nct = (ncol + TC - 1) / TC;
  const int rt = lb / nct;
  const int m = tiles[2 * rt] >> 1;
  const int row0 = tiles[2 * rt + 1];
  const int col0 = (lb - rt * nct) * TC;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave / WC) * (TR / WR), wc = (wave % WC) * (TC / WC);
  const int li = lane & 15, lk = lane >> 4;
  const size_t gbase = (size_t)m * fourier_pitch<E>(nlat, ncol);

  typename MM::acc_t acc[2][BI][BJ];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j) acc[q][i][j] = MM::zero();

  // k-slabs: the even rows' slabs, then the odd rows'
  const int roff0 = rowoff[2 * m], K0 = rowoff[2 * m + 1] - roff0;
  const int roff1 = rowoff[2 * m + 1], K1 = rowoff[2 * m + 2] - roff1;
  const int ns0 = (K0 + TK - 1) / TK, ns1 = (K1 + TK - 1) / TK;
  const int nslab = ns0 + ns1;
  E ra[NA], rb[NB];
  auto fetch = [&](int sl) {
    const bool second = sl >= ns0;
    const int roff = second ? roff1 : roff0;
    const int K = second ? K1 : K0;
    const int k0 = (second ? sl - ns0 : sl) * TK;
#pragma unroll
    for (int e4 = 0; e4 < NA; ++e4) {
      const int e = tid + e4 * 256;
      const int kk = e / TR, rr = e % TR;              // lanes along the latitudes
      const int k = k0 + kk, r = row0 + rr;
      ra[e4] = (k < K && r < nlat2) ? T[(size_t)(roff + k) * nlat2 + r] : E(0);
    }
#pragma unroll
    for (int e4 = 0; e4 < NB; ++e4) {
      const int e = tid + e4 * 256;
      const int kk = e / TC, cc = e % TC;
      const int k = k0 + kk, c = col0 + cc;
      rb[e4] = (k < K && c < ncol) ? S[(size_t)(roff + k) * ncol + c] : E(0);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int e4 = 0; e4 < NA; ++e4) {
      const int e = tid + e4 * 256;
      As[buf][(e / TR) * LDA + (e % TR)] = ra[e4];
    }
#pragma unroll
    for (int e4 = 0; e4 < NB; ++e4) {
      const int e = tid + e4 * 256;
      Bs[buf][(e / TC) * LDB + (e % TC)] = rb[e4];
    }
  };
  auto mma = [&](int cur, typename MM::acc_t (&ac)[BI][BJ]) {
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      E a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = As[cur][(ks + lk) * LDA + wr + 16 * i + li];
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = Bs[cur][(ks + lk) * LDB + wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) ac[i][j] = MM::mma(a[i], b[j], ac[i][j]);
    }
  };

  if (nslab > 0) {
    fetch(0);
    stash(0);
  }
  __syncthreads();
  // parity 0 slabs (the last one prefetches parity 1's first), then parity 1
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    for (int sl = q ? ns0 : 0; sl < (q ? nslab : ns0); ++sl) {
      const int cur = sl & 1;
      if (sl + 1 < nslab) fetch(sl + 1);
      mma(cur, acc[q]);
      if (sl + 1 < nslab) stash(cur ^ 1);
      __syncthreads();
    }
  }
  // ---- store (result layout of Mma<E>) ----
#pragma unroll
  for (int bi = 0; bi < BI; ++bi) {
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      const int c = col0 + wc + bj * 16 + li;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = row0 + wr + bi * 16 + MM::row(lk, i);
        if (r < nlat2 && c < ncol) {
          const E e = acc[0][bi][bj][i], o = acc[1][bi][bj][i];
          F[gbase + (size_t)r * ncol + c] = e + o;
          F[gbase + (size_t)(nlat - 1 - r) * ncol + c] = e - o;
        }
      }
    }
  }
}

// Analysis tile: TR2 = 32 rows of each parity of one m (64 rows in all) x TC
// columns.  Both parities contract over the same northern latitudes k with
// B_E = G(k) + G(nlat-1-k) and B_O = G(k) - G(nlat-1-k), formed from one load
// of each pair.  The row-wave groups of the first half of the tile take the
// even rows, the others the odd rows.  Per output element the matrix cores
// consume k in steps of 4 in increasing order, as in every other shape.
template <typename E, int TC, int TK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_legendre_anal(
    const E* __restrict__ Tt, const int* __restrict__ rowoff, const int* __restrict__ tiles,
    const E* __restrict__ G, E* __restrict__ Q, int nlat, int nlat2, int ncol, int nrows) {
  using MM = Mma<E>;
  constexpr int TR2 = 32, TR = 2 * TR2;
  constexpr int LDA = TR + 2, LDB = TC + 2;
  constexpr int NA = TK * TR / 256;                  // A elements per thread per slab
  constexpr int NB = TK * TC / 256;                  // G pairs per thread per slab
  constexpr int WC = TC >= 64 ? 2 : 1;               // waves across columns
  constexpr int WR = 4 / WC;                         // waves across rows
  constexpr int BI = TR / WR / 16, BJ = TC / WC / 16;
  static_assert(BI >= 1 && BJ >= 1 && NA >= 1 && NB >= 1 && (TR / WR) <= TR2, "tile shape");
  // one LDS slab (the next one is held in registers while the current one
  // is consumed): four workgroups per CU instead of three
  __shared__ E As[TK * LDA];
  __shared__ E Bs[2][TK * LDB];                      // [parity]

  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int nct = (ncol + TC - 1) / TC;
  const int rt = lb / nct;
  const int m = tiles[2 * rt] >> 1;
  const int row0 = tiles[2 * rt + 1];
  const int col0 = (lb - rt * nct) * TC;
  const int roffE = rowoff[2 * m], cntE = rowoff[2 * m + 1] - roffE;
  const int roffO = rowoff[2 * m + 1], cntO = rowoff[2 * m + 2] - roffO;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave / WC) * (TR / WR), wc = (wave % WC) * (TC / WC);
  const int par = wr >= TR2;                         // uniform per wave
  const int li = lane & 15, lk = lane >> 4;
  const size_t gbase = (size_t)m * fourier_pitch<E>(nlat, ncol);

  typename MM::acc_t acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = MM::zero();

  // the next slab's loads stay in flight across the current slab's matrix
  // products: fetch only issues them (raw north and south values), and the
  // parity sums are formed when the slab is stashed
  E ra[NA], rgn[NB], rgs[NB];
  bool pa[NA], pb[NB];
  // loads at clamped indices, issued without branches (32-bit offsets within
  // the table and within m's Fourier rows), out-of-tile elements zeroed
  static_assert(256 % TR == 0 && 256 % TC == 0, "a thread keeps its row and column");
  const int ri = tid % TR;
  const bool odd = ri >= TR2;
  const int ar = row0 + (odd ? ri - TR2 : ri), acnt = odd ? cntO : cntE;
  const bool aok = ar < acnt;
  const int acol = (odd ? roffO : roffE) + (aok ? ar : acnt - 1);
  const int bc = col0 + tid % TC;
  const bool bok = bc < ncol;
  const int bcl = bok ? bc : ncol - 1;
  const E* Gm = G + gbase;
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e4 = 0; e4 < NA; ++e4) {
      const int k = k0 + (tid + e4 * 256) / TR;
      const int kc = k < nlat2 ? k : nlat2 - 1;
      ra[e4] = Tt[kc * nrows + acol];
      pa[e4] = k < nlat2 && aok;
    }
#pragma unroll
    for (int e4 = 0; e4 < NB; ++e4) {
      const int k = k0 + (tid + e4 * 256) / TC;
      const int kc = k < nlat2 ? k : nlat2 - 1;
      rgn[e4] = Gm[kc * ncol + bcl];
      rgs[e4] = Gm[(nlat - 1 - kc) * ncol + bcl];
      pb[e4] = k < nlat2 && bok;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int e4 = 0; e4 < NA; ++e4) {
      const int e = tid + e4 * 256;
      As[(e / TR) * LDA + (e % TR)] = pa[e4] ? ra[e4] : E(0);
    }
#pragma unroll
    for (int e4 = 0; e4 < NB; ++e4) {
      const int e = tid + e4 * 256;
      const E gn = pb[e4] ? rgn[e4] : E(0), gs = pb[e4] ? rgs[e4] : E(0);
      Bs[0][(e / TC) * LDB + (e % TC)] = gn + gs;
      Bs[1][(e / TC) * LDB + (e % TC)] = gn + E(-1) * gs;
    }
  };
  const int nslab = (nlat2 + TK - 1) / TK;
  fetch(0);
  stash();
  __syncthreads();
  for (int sl = 0; sl < nslab; ++sl) {
    if (sl + 1 < nslab) fetch((sl + 1) * TK);
    const E* bs = Bs[par];
#pragma unroll
    for (int ks = 0; ks < TK; ks += 4) {
      E a[BI], b[BJ];
#pragma unroll
      for (int i = 0; i < BI; ++i) a[i] = As[(ks + lk) * LDA + wr + 16 * i + li];
#pragma unroll
      for (int j = 0; j < BJ; ++j) b[j] = bs[(ks + lk) * LDB + wc + 16 * j + li];
#pragma unroll
      for (int i = 0; i < BI; ++i)
#pragma unroll
        for (int j = 0; j < BJ; ++j) acc[i][j] = MM::mma(a[i], b[j], acc[i][j]);
    }
    if (sl + 1 < nslab) {
      __syncthreads();                               // every wave has read the slab
      stash();
    }
    __syncthreads();
  }
  const int roff = par ? roffO : roffE, cnt = par ? cntO : cntE;
  const int wrp = wr - par * TR2;                    // row offset within the parity
#pragma unroll
  for (int bi = 0; bi < BI; ++bi) {
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      const int c = col0 + wc + bj * 16 + li;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = row0 + wrp + bi * 16 + MM::row(lk, i);
        if (r < cnt && c < ncol) Q[(size_t)(roff + r) * ncol + c] = acc[bi][bj][i];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split-BF16 variant (PINT_LEG_BF16X3): FP32 operands x = hi + lo with hi the
// BF16 rounding of x and lo the BF16 rounding of x - hi (exact in FP32);
// each product sums lo_a hi_b + hi_a lo_b + hi_a hi_b on the BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16) with FP32 accumulation, dropping lo_a lo_b
// (three products: Henry, Tang and Heinecke, ARITH 2019).  The split is made
// while a slab is staged in LDS.  One instruction consumes k in blocks of 32,
// lane l holding the 8 values k = 8(l/16) + e of row (A) or column (B) l%16,
// so LDS holds each row and column k-contiguous (one 16-byte read per lane
// and operand).  Slabs start at k = 0 of each parity for every tile shape:
// the k-order of every output element is independent of the batch.
// ---------------------------------------------------------------------------
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ inline void split8(const float (&x)[8], v8bf& hi, v8bf& lo) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const __bf16 h = (__bf16)x[e];
    hi[e] = h;
    lo[e] = (__bf16)(x[e] - (float)h);
  }
}

__device__ inline v4f mma3(v8bf ah, v8bf al, v8bf bh, v8bf bl, v4f c) {
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, c, 0, 0, 0);
  c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, c, 0, 0, 0);
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, c, 0, 0, 0);
}

constexpr int kBfTK = 32;                 // k per slab (one instruction)
constexpr int kBfKG = kBfTK / 8;          // 8-value groups per row per slab
constexpr int kBfLD = kBfKG + 1;          // padded LDS row, in 8-value groups

// Synthesis tile as k_legendre_synth: TR = 64 latitudes x TC columns, both
// parities of one m, epilogue E +- O.  One LDS slab, the next one held in
// registers while the current one is consumed.
template <int TC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_legendre_synth_bf3(
    const float* __restrict__ T, const int* __restrict__ rowoff, const int* __restrict__ tiles,
    const float* __restrict__ S, float* __restrict__ F, int nlat, int nlat2, int ncol) {
  constexpr int TR = 64;
  constexpr int WC = TC >= 64 ? 2 : 1;               // waves across columns
  constexpr int WR = 4 / WC;                         // waves across rows
  constexpr int BI = TR / WR / 16, BJ = TC / WC / 16;
  static_assert(BI >= 1 && BJ >= 1 && TR * kBfKG == 256 && TC * kBfKG <= 256, "tile shape");
  __shared__ v8bf Ah[TR * kBfLD], Al[TR * kBfLD];
  __shared__ v8bf Bh[TC * kBfLD], Bl[TC * kBfLD];

  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int nct = (ncol + TC - 1) / TC;
  const int rt = lb / nct;
  const int m = tiles[2 * rt] >> 1;
  const int row0 = tiles[2 * rt + 1];
  const int col0 = (lb - rt * nct) * TC;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave / WC) * (TR / WR), wc = (wave % WC) * (TC / WC);
  const int li = lane & 15, lk = lane >> 4;
  const size_t gbase = (size_t)m * fourier_pitch<float>(nlat, ncol);

  v4f acc[2][BI][BJ];
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j) acc[q][i][j] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};

  const int roff0 = rowoff[2 * m], K0 = rowoff[2 * m + 1] - roff0;
  const int roff1 = rowoff[2 * m + 1], K1 = rowoff[2 * m + 2] - roff1;
  const int ns0 = (K0 + kBfTK - 1) / kBfTK, ns1 = (K1 + kBfTK - 1) / kBfTK;
  const int nslab = ns0 + ns1;
  // loader roles: A row ra_r (lanes along latitudes), k-group ra_g; B column
  // rb_c (lanes along columns), k-group rb_g, for the first TC * 4 threads
  const int ra_r = tid % TR, ra_g = tid / TR;
  const bool bload = tid < TC * kBfKG;
  const int rb_c = tid % TC, rb_g = tid / TC;
  float xa[8], xb[8];
  auto fetch = [&](int sl) {
    const bool second = sl >= ns0;
    const int roff = second ? roff1 : roff0;
    const int K = second ? K1 : K0;
    const int k0 = (second ? sl - ns0 : sl) * kBfTK + 8 * ra_g;
    const int r = row0 + ra_r;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + e;
      xa[e] = (k < K && r < nlat2) ? T[(size_t)(roff + k) * nlat2 + r] : 0.0f;
    }
    if (bload) {
      const int kb = (second ? sl - ns0 : sl) * kBfTK + 8 * rb_g;
      const int c = col0 + rb_c;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = kb + e;
        xb[e] = (k < K && c < ncol) ? S[(size_t)(roff + k) * ncol + c] : 0.0f;
      }
    }
  };
  auto stash = [&]() {
    v8bf h, l;
    split8(xa, h, l);
    Ah[ra_r * kBfLD + ra_g] = h;
    Al[ra_r * kBfLD + ra_g] = l;
    if (bload) {
      split8(xb, h, l);
      Bh[rb_c * kBfLD + rb_g] = h;
      Bl[rb_c * kBfLD + rb_g] = l;
    }
  };
  auto mma = [&](v4f (&ac)[BI][BJ]) {
    v8bf ah[BI], al[BI], bh[BJ], bl[BJ];
#pragma unroll
    for (int i = 0; i < BI; ++i) {
      ah[i] = Ah[(wr + 16 * i + li) * kBfLD + lk];
      al[i] = Al[(wr + 16 * i + li) * kBfLD + lk];
    }
#pragma unroll
    for (int j = 0; j < BJ; ++j) {
      bh[j] = Bh[(wc + 16 * j + li) * kBfLD + lk];
      bl[j] = Bl[(wc + 16 * j + li) * kBfLD + lk];
    }
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j) ac[i][j] = mma3(ah[i], al[i], bh[j], bl[j], ac[i][j]);
  };

  if (nslab > 0) {
    fetch(0);
    stash();
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    for (int sl = q ? ns0 : 0; sl < (q ? nslab : ns0); ++sl) {
      if (sl + 1 < nslab) fetch(sl + 1);
      mma(acc[q]);
      if (sl + 1 < nslab) {
        __syncthreads();                             // every wave has read the slab
        stash();
      }
      __syncthreads();
    }
  }
  // store: register i of lane l holds D[4(l/16) + i][l%16]
#pragma unroll
  for (int bi = 0; bi < BI; ++bi) {
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      const int c = col0 + wc + bj * 16 + li;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = row0 + wr + bi * 16 + 4 * lk + i;
        if (r < nlat2 && c < ncol) {
          const float e = acc[0][bi][bj][i], o = acc[1][bi][bj][i];
          F[gbase + (size_t)r * ncol + c] = e + o;
          F[gbase + (size_t)(nlat - 1 - r) * ncol + c] = e - o;
        }
      }
    }
  }
}

// Analysis tile as k_legendre_anal: 32 rows of each parity x TC columns,
// contraction over the northern latitudes with B_E = G(k) + G(nlat-1-k),
// B_O = G(k) - G(nlat-1-k).  One LDS slab (the next one is held in registers
// while the current one is consumed) keeps four workgroups per CU.
template <int TC>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_legendre_anal_bf3(
    const float* __restrict__ Tt, const int* __restrict__ rowoff, const int* __restrict__ tiles,
    const float* __restrict__ G, float* __restrict__ Q, int nlat, int nlat2, int ncol,
    int nrows) {
  constexpr int TR2 = 32, TR = 2 * TR2;
  constexpr int WC = TC >= 32 ? TC / 32 : 1;
  constexpr int WR = 4 / WC;
  constexpr int BI = TR / WR / 16, BJ = TC / WC / 16;
  static_assert(BI >= 1 && BJ >= 1 && (TR / WR) <= TR2 && TR * kBfKG == 256 &&
                    TC * kBfKG <= 256, "tile shape");
  __shared__ v8bf Ah[TR * kBfLD], Al[TR * kBfLD];
  __shared__ v8bf Bh[2][TC * kBfLD], Bl[2][TC * kBfLD];         // [parity]

  const int lb = xcd_remap(blockIdx.x, gridDim.x);
  const int nct = (ncol + TC - 1) / TC;
  const int rt = lb / nct;
  const int m = tiles[2 * rt] >> 1;
  const int row0 = tiles[2 * rt + 1];
  const int col0 = (lb - rt * nct) * TC;
  const int roffE = rowoff[2 * m], cntE = rowoff[2 * m + 1] - roffE;
  const int roffO = rowoff[2 * m + 1], cntO = rowoff[2 * m + 2] - roffO;
  const int tid = threadIdx.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int wr = (wave / WC) * (TR / WR), wc = (wave % WC) * (TC / WC);
  const int par = wr >= TR2;                         // uniform per wave
  const int li = lane & 15, lk = lane >> 4;
  const size_t gbase = (size_t)m * fourier_pitch<float>(nlat, ncol);

  v4f acc[BI][BJ];
#pragma unroll
  for (int i = 0; i < BI; ++i)
#pragma unroll
    for (int j = 0; j < BJ; ++j) acc[i][j] = (v4f){0.0f, 0.0f, 0.0f, 0.0f};

  const int ra_r = tid % TR, ra_g = tid / TR;
  const bool a_odd = ra_r >= TR2;
  const int a_row = row0 + (a_odd ? ra_r - TR2 : ra_r);
  const bool a_ok = a_row < (a_odd ? cntO : cntE);
  const int a_off = (a_odd ? roffO : roffE) + a_row;
  const bool bload = tid < TC * kBfKG;
  const int rb_c = tid % TC, rb_g = tid / TC;
  float xa[8], xn[8], xs[8];   // raw north / south values: sums formed at stash
  auto fetch = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = k0 + 8 * ra_g + e;
      xa[e] = (a_ok && k < nlat2) ? Tt[(size_t)k * nrows + a_off] : 0.0f;
    }
    if (bload) {
      const int c = col0 + rb_c;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = k0 + 8 * rb_g + e;
        float gn = 0.0f, gs = 0.0f;
        if (k < nlat2 && c < ncol) {
          gn = G[gbase + (size_t)k * ncol + c];
          gs = G[gbase + (size_t)(nlat - 1 - k) * ncol + c];
        }
        xn[e] = gn;
        xs[e] = gs;
      }
    }
  };
  auto stash = [&]() {
    v8bf h, l;
    split8(xa, h, l);
    Ah[ra_r * kBfLD + ra_g] = h;
    Al[ra_r * kBfLD + ra_g] = l;
    if (bload) {
      float xe[8], xo[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        xe[e] = xn[e] + xs[e];
        xo[e] = xn[e] - xs[e];
      }
      split8(xe, h, l);
      Bh[0][rb_c * kBfLD + rb_g] = h;
      Bl[0][rb_c * kBfLD + rb_g] = l;
      split8(xo, h, l);
      Bh[1][rb_c * kBfLD + rb_g] = h;
      Bl[1][rb_c * kBfLD + rb_g] = l;
    }
  };
  const int nslab = (nlat2 + kBfTK - 1) / kBfTK;
  fetch(0);
  stash();
  __syncthreads();
  for (int sl = 0; sl < nslab; ++sl) {
    if (sl + 1 < nslab) fetch((sl + 1) * kBfTK);
    v8bf ah[BI], al[BI], bh[BJ], bl[BJ];
#pragma unroll
    for (int i = 0; i < BI; ++i) {
      ah[i] = Ah[(wr + 16 * i + li) * kBfLD + lk];
      al[i] = Al[(wr + 16 * i + li) * kBfLD + lk];
    }
#pragma unroll
    for (int j = 0; j < BJ; ++j) {
      bh[j] = Bh[par][(wc + 16 * j + li) * kBfLD + lk];
      bl[j] = Bl[par][(wc + 16 * j + li) * kBfLD + lk];
    }
#pragma unroll
    for (int i = 0; i < BI; ++i)
#pragma unroll
      for (int j = 0; j < BJ; ++j) acc[i][j] = mma3(ah[i], al[i], bh[j], bl[j], acc[i][j]);
    if (sl + 1 < nslab) {
      __syncthreads();                               // every wave has read the slab
      stash();
    }
    __syncthreads();
  }
  const int roff = par ? roffO : roffE, cnt = par ? cntO : cntE;
  const int wrp = wr - par * TR2;
#pragma unroll
  for (int bi = 0; bi < BI; ++bi) {
#pragma unroll
    for (int bj = 0; bj < BJ; ++bj) {
      const int c = col0 + wc + bj * 16 + li;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = row0 + wrp + bi * 16 + 4 * lk + i;
        if (r < cnt && c < ncol) Q[(size_t)(roff + r) * ncol + c] = acc[bi][bj][i];
      }
    }
  }
}

// Launch shapes.  Every shape consumes k in the same order (steps of 4,
// increasing, per parity), so all give bitwise the same results and the
// choice between them is a matter of speed only: narrow column tiles (16)
// for launches of up to two states (synthesis) or four (analysis), 64 or 128
// otherwise, and a k-slab depth TK of 16 or 32, chosen per plan and launch
// class by the autotuner (tune_legendre) or left at the default (variant 0).
enum { kClassSmall = 0, kClassLarge = 1 };
static int gemm_class(int ncol) { return ncol <= 32 ? kClassSmall : kClassLarge; }

template <typename E>
static void launch_synth(Plan& p, const E* T, const E* S, E* F, int ncol, hipStream_t s) {
  const int cls = gemm_class(ncol);
  const int v = p.gemm_variant[0][cls];
  if (cls == kClassSmall) {
    dim3 grid(((ncol + 15) / 16) * p.syn_tiles.count);
    if (v == 1)
      hipLaunchKernelGGL((k_legendre_synth<E, kGemmTR, 16, 32>), grid, dim3(256), 0, s, T,
                         p.rowoff, p.syn_tiles.dev, S, F, p.nlat, p.nlat2, ncol);
    else
      hipLaunchKernelGGL((k_legendre_synth<E, kGemmTR, 16, kGemmTK>), grid, dim3(256), 0, s, T,
                         p.rowoff, p.syn_tiles.dev, S, F, p.nlat, p.nlat2, ncol);
  } else if (v == 1) {
    dim3 grid(((ncol + 127) / 128) * p.syn_tiles.count);
    hipLaunchKernelGGL((k_legendre_synth<E, kGemmTR, 128, kGemmTK>), grid, dim3(256), 0, s, T,
                       p.rowoff, p.syn_tiles.dev, S, F, p.nlat, p.nlat2, ncol);
  } else {
    dim3 grid(((ncol + 63) / 64) * p.syn_tiles.count);
    hipLaunchKernelGGL((k_legendre_synth<E, kGemmTR, 64, kGemmTK>), grid, dim3(256), 0, s, T,
                       p.rowoff, p.syn_tiles.dev, S, F, p.nlat, p.nlat2, ncol);
  }
}

template <typename E>
static void launch_anal(Plan& p, const E* Tt, const E* G, E* Q, int ncol, hipStream_t s) {
  const int cls = gemm_class(ncol);
  const int v = p.gemm_variant[1][cls];
  if (cls == kClassSmall) {
    dim3 grid(((ncol + 15) / 16) * p.ana_tiles.count);
    if (v == 1)
      hipLaunchKernelGGL((k_legendre_anal<E, 16, 32>), grid, dim3(256), 0, s, Tt, p.rowoff,
                         p.ana_tiles.dev, G, Q, p.nlat, p.nlat2, ncol, p.nrows);
    else
      hipLaunchKernelGGL((k_legendre_anal<E, 16, kGemmTK>), grid, dim3(256), 0, s, Tt, p.rowoff,
                         p.ana_tiles.dev, G, Q, p.nlat, p.nlat2, ncol, p.nrows);
  } else if (v == 2) {
    dim3 grid(((ncol + 127) / 128) * p.ana_tiles.count);
    hipLaunchKernelGGL((k_legendre_anal<E, 128, kGemmTK>), grid, dim3(256), 0, s, Tt, p.rowoff,
                       p.ana_tiles.dev, G, Q, p.nlat, p.nlat2, ncol, p.nrows);
  } else {
    dim3 grid(((ncol + 63) / 64) * p.ana_tiles.count);
    if (v == 1)
      hipLaunchKernelGGL((k_legendre_anal<E, 64, 32>), grid, dim3(256), 0, s, Tt, p.rowoff,
                         p.ana_tiles.dev, G, Q, p.nlat, p.nlat2, ncol, p.nrows);
    else
      hipLaunchKernelGGL((k_legendre_anal<E, 64, kGemmTK>), grid, dim3(256), 0, s, Tt, p.rowoff,
                         p.ana_tiles.dev, G, Q, p.nlat, p.nlat2, ncol, p.nrows);
  }
}

// Variants per (transform, launch class): few states -- k-slabs of 16 or 32;
// many states -- synthesis with 64- or 128-column tiles (k-slabs of 16: 32
// would need more than 64 KiB of LDS), analysis with 64 columns and k-slabs
// of 16 or 32, or 128 columns (the table read half as often).
static int gemm_variants(int kind, int cls) {
  return cls == kClassSmall ? 2 : (kind == 0 ? 2 : 3);
}

static void launch_synth_bf3(Plan& p, int ncol, hipStream_t s) {
  const float* T = p.ptab32;
  const float* S = reinterpret_cast<const float*>(p.S);
  float* F = reinterpret_cast<float*>(p.F);
  if (ncol <= 32) {
    dim3 grid(((ncol + 15) / 16) * p.syn_tiles.count);
    hipLaunchKernelGGL(k_legendre_synth_bf3<16>, grid, dim3(256), 0, s, T, p.rowoff,
                       p.syn_tiles.dev, S, F, p.nlat, p.nlat2, ncol);
  } else {
    dim3 grid(((ncol + 63) / 64) * p.syn_tiles.count);
    hipLaunchKernelGGL(k_legendre_synth_bf3<64>, grid, dim3(256), 0, s, T, p.rowoff,
                       p.syn_tiles.dev, S, F, p.nlat, p.nlat2, ncol);
  }
}

static void launch_anal_bf3(Plan& p, int ncol, hipStream_t s) {
  const float* Tt = p.ptabT32;
  const float* G = reinterpret_cast<const float*>(p.G);
  float* Q = reinterpret_cast<float*>(p.Q);
  if (ncol <= 32) {
    dim3 grid(((ncol + 15) / 16) * p.ana_tiles.count);
    hipLaunchKernelGGL(k_legendre_anal_bf3<16>, grid, dim3(256), 0, s, Tt, p.rowoff,
                       p.ana_tiles.dev, G, Q, p.nlat, p.nlat2, ncol, p.nrows);
  } else {
    dim3 grid(((ncol + 63) / 64) * p.ana_tiles.count);
    hipLaunchKernelGGL(k_legendre_anal_bf3<64>, grid, dim3(256), 0, s, Tt, p.rowoff,
                       p.ana_tiles.dev, G, Q, p.nlat, p.nlat2, ncol, p.nrows);
  }
}

pint_status legendre_synth(Plan& p, int B, int nf, int prec, hipStream_t s) {
  ProfScope ps(p, PK_SYNTH, nf == kSynFields ? B : -B, s);
  const int ncol = 2 * nf * B;
  if (prec == PINT_LEG_BF16X3)
    launch_synth_bf3(p, ncol, s);
  else if (prec == PINT_LEG_FP32)
    launch_synth<float>(p, p.ptab32, reinterpret_cast<const float*>(p.S),
                        reinterpret_cast<float*>(p.F), ncol, s);
  else
    launch_synth<double>(p, p.ptab, p.S, p.F, ncol, s);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

pint_status legendre_anal(Plan& p, int B, int nf, int prec, hipStream_t s) {
  ProfScope ps(p, PK_ANAL, nf == kAnaFields ? B : -B, s);
  const int ncol = 2 * nf * B;
  if (prec == PINT_LEG_BF16X3)
    launch_anal_bf3(p, ncol, s);
  else if (prec == PINT_LEG_FP32)
    launch_anal<float>(p, p.ptabT32, reinterpret_cast<const float*>(p.G),
                       reinterpret_cast<float*>(p.Q), ncol, s);
  else
    launch_anal<double>(p, p.ptabT, p.G, p.Q, ncol, s);
  PINT_HIP(hipGetLastError());
  return PINT_OK;
}

// Autotuner: for each transform and launch class, time every variant on the
// plan's workspace (launches of `states` states: the classes' batch sizes of
// the coming work) and keep the fastest.  The variants give bitwise the same
// results, so the choice never changes an answer.  Synchronises `s`.
pint_status tune_legendre(Plan& p, const int (&states)[2], hipStream_t s) {
  if (p.prec == PINT_LEG_BF16X3) return PINT_OK;   // one shape per class there
  hipEvent_t e0, e1;
  PINT_HIP(hipEventCreate(&e0));
  PINT_HIP(hipEventCreate(&e1));
  pint_status st = PINT_OK;
  for (int kind = 0; kind < 2 && st == PINT_OK; ++kind) {
    for (int cls = 0; cls < 2 && st == PINT_OK; ++cls) {
      const int B = states[cls];
      if (B < 1 || B > p.max_batch) continue;
      const int nf = kind == 0 ? kSynFields : kAnaFields;
      if (gemm_class(2 * nf * B) != cls) continue;
      int best = 0;
      float best_ms = 0.0f;
      for (int v = 0; v < gemm_variants(kind, cls) && st == PINT_OK; ++v) {
        p.gemm_variant[kind][cls] = v;
        float ms = 0.0f;
        for (int rep = 0; rep < 4 && st == PINT_OK; ++rep) {   // first one warms up
          if (rep == 1 && hipEventRecord(e0, s) != hipSuccess) st = PINT_E_HIP;
          if (st == PINT_OK)
            st = kind == 0 ? legendre_synth(p, B, nf, p.prec, s) : legendre_anal(p, B, nf, p.prec, s);
        }
        if (st == PINT_OK && (hipEventRecord(e1, s) != hipSuccess ||
                              hipEventSynchronize(e1) != hipSuccess ||
                              hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
          st = PINT_E_HIP;
        if (st == PINT_OK && (v == 0 || ms < best_ms)) {
          best = v;
          best_ms = ms;
        }
      }
      p.gemm_variant[kind][cls] = best;
      p.gemm_tuned_ms[kind][cls] = best_ms / 3.0f;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == PINT_E_HIP) set_error("timing the Legendre GEMM variants failed");
  return st;
}

}  // namespace pint
