// Left-looking Cholesky of the large sizes by block panels, as a sequence of
// launches that each cover the whole batch.  For the panel of rows
// [k0, k0 + NB) of the upper factor (the partitioned form of the paper's
// Cholesky, Fig. 2a, taken by block rows):
//
//   A(k0:k0+NB, k0:n) -= X(0:k0, k0:k0+NB)^T X(0:k0, k0:n)    panel update
//   X(k0:k0+NB, k0:k0+NB) = chol(A(k0:k0+NB, k0:k0+NB))         diagonal block
//   X(k0:k0+NB, k0+NB:n) = X_kk^{-T} A(k0:k0+NB, k0+NB:n)       panel solve
//
// The update carries almost all of the n^3/3 flops.  It runs as one batched
// product over all instances (k_bgemm_chol: 64 x 64 output blocks per
// workgroup, 16-deep operand panels staged in LDS, FP64 matrix cores),
// instead of tile products inside one workgroup per instance: a 16-wave
// instance workgroup re-reads every operand tile from memory and keeps one
// compute unit busy per instance.  The diagonal block uses the in-place
// Cholesky kernel (order NB, four waves) on pointers into the caller's
// matrices, and the panel solve runs many 16-column tiles per instance side
// by side (k_panel_trsm).
// Only the upper triangle is read or written.
#include <cstdio>
#include <cstdlib>

#include "tla_inplace.hpp"
#include "tla_host.h"

namespace tla {

constexpr int kPanelNB = 128;  // panel height

namespace {

#define PN_HIP(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      if (getenv("TLA_LOG")) fprintf(stderr, "tla: %s failed: %s\n", #x, hipGetErrorString(e_)); \
      return TLA_E_HIP;                                                             \
    }                                                                               \
  } while (0)

struct PanelArgs {
  int batch, n_max, k0, nb;
  const int* n;          // the instance's order, 0 when it is invalid or has failed validation
  double* const* x;      // the caller's matrices
  const int* ld;
};

// C(i, j) -= sum_k X(k, k0 + i) X(k, k0 + j) over k < k0, for
// 0 <= i < min(nb, n - k0), i <= j < n - k0 (upper triangle only).
// Grid (column blocks of 128, row blocks of 128, instances), 4 waves.
constexpr int kBk = 16;  // depth of the staged operand panels

// ---- batched product core: acc += A B for one BM x BM output block
// (BM = 64 or 128).  A (BM x K) is read either k-contiguous (element (i, k)
// at A[k + i lda], AK) or row-contiguous (A[i + k lda]); B (K x BM)
// k-contiguous (B[k + j ldb]).  Rows i >= mr of A and columns j >= mc of B
// read as zero; K is a multiple of 16.  256 threads: wave w accumulates the
// quadrant (w >> 1, w & 1) as TW x TW tiles of 16 x 16 on the FP64 matrix
// cores; 16-deep panels of A and B are staged in LDS and the next pair is
// loaded into registers while the current one is multiplied.
typedef double d4v __attribute__((ext_vector_type(4)));

template <int BM>
struct Core {
  static constexpr int TW = BM / 32, LD = BM + 4, E = BM / 16;  // tiles per wave dim, LDS stride, loads per thread
};

template <int BM, bool AK>
TLA_DI void bgemm_core(d4v (&acc)[BM / 32][BM / 32], const gbl_t<double>* A, int lda, const gbl_t<double>* B,
                       int ldb, int K, int mr, int mc, lds_t<double>* sA, lds_t<double>* sB) {
  constexpr int TW = Core<BM>::TW, LD = Core<BM>::LD, E = Core<BM>::E, RS = 256 / BM;
  const int t = threadIdx.x, l = lane_id(), w = wave_id();
  const int wr = (w >> 1) * (BM / 2), wc = (w & 1) * (BM / 2), i16 = l & 15, kq = l >> 4;
  double ra[E], rb[E];
  // element r of this thread: A row (t >> 4) + 16 r at k = t & 15 (AK) or row
  // t % BM at k = t / BM + RS r; B column (t >> 4) + 16 r at k = t & 15.
  // One base pointer per operand; lanes outside the block load nothing.
  const gbl_t<double>* pa = AK ? A + (t & 15) + (size_t)(t >> 4) * lda : A + (t % BM) + (size_t)(t / BM) * lda;
  const gbl_t<double>* pb = B + (t & 15) + (size_t)(t >> 4) * ldb;
  const size_t sa = AK ? (size_t)16 * lda : (size_t)RS * lda, sb = (size_t)16 * ldb;
  auto fetch = [&](int kt) {
    const size_t ka = AK ? (size_t)kt : (size_t)kt * lda;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const bool ina = AK ? (t >> 4) + 16 * r < mr : (t % BM) < mr;
      ra[r] = ina ? pa[ka + r * sa] : 0.0;
      rb[r] = (t >> 4) + 16 * r < mc ? pb[kt + r * sb] : 0.0;
    }
  };
  if (K <= 0) return;
  fetch(0);
  for (int kt = 0; kt < K; kt += kBk) {
    __syncthreads();
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int e = t + 256 * r;
      if constexpr (AK) sA[(e & 15) * LD + (e >> 4)] = ra[r];
      else sA[(e / BM) * LD + (e % BM)] = ra[r];
      sB[(e & 15) * LD + (e >> 4)] = rb[r];
    }
    __syncthreads();
    if (kt + kBk < K) fetch(kt + kBk);
#pragma unroll
    for (int k4 = 0; k4 < 4; ++k4) {
      const int kr = (4 * k4 + kq) * LD;
      double fa[TW], fb[TW];
#pragma unroll
      for (int a = 0; a < TW; ++a) fa[a] = sA[kr + wr + 16 * a + i16];
#pragma unroll
      for (int c = 0; c < TW; ++c) fb[c] = sB[kr + wc + 16 * c + i16];
#pragma unroll
      for (int a = 0; a < TW; ++a)
#pragma unroll
        for (int c = 0; c < TW; ++c) acc[a][c] = __builtin_amdgcn_mfma_f64_16x16x4f64(fa[a], fb[c], acc[a][c], 0, 0, 0);
    }
  }
}

template <int TW>
TLA_DI void zero_acc(d4v (&acc)[TW][TW]) {
#pragma unroll
  for (int a = 0; a < TW; ++a)
#pragma unroll
    for (int c = 0; c < TW; ++c) acc[a][c] = d4v{0.0, 0.0, 0.0, 0.0};
}

constexpr int kCholBM = 64;  // (128 measured 8% slower: too few blocks late in the factorisation)

__global__ __launch_bounds__(256) void k_bgemm_chol(PanelArgs g) {
  constexpr int BM = kCholBM, TW = Core<BM>::TW;
  __shared__ double sA[kBk * Core<BM>::LD];
  __shared__ double sB[kBk * Core<BM>::LD];
  const int b = blockIdx.z;
  const int n = g.n[b];
  const int k0 = g.k0;
  if (n <= k0) return;
  const int M = n - k0 < g.nb ? n - k0 : g.nb, N = n - k0;
  const int i0 = blockIdx.y * BM, j0 = blockIdx.x * BM;
  if (i0 >= M || j0 >= N || i0 > j0 + BM - 1) return;  // nothing of the upper triangle here
  const int ld = g.ld[b];
  const gbl_t<double>* X = to_gbl(static_cast<const double*>(g.x[b]));
  d4v acc[TW][TW];
  zero_acc<TW>(acc);
  // A(i, k) = X(k, k0 + i0 + i), B(k, j) = X(k, k0 + j0 + j), k < k0
  bgemm_core<BM, true>(acc, X + (size_t)(k0 + i0) * ld, ld, X + (size_t)(k0 + j0) * ld, ld, k0, M - i0, N - j0,
                       to_lds(sA), to_lds(sB));
  gbl_t<double>* C = to_gbl(g.x[b]);
  const int l = lane_id(), w = wave_id(), wr = (w >> 1) * (BM / 2), wc = (w & 1) * (BM / 2);
#pragma unroll
  for (int a = 0; a < TW; ++a)
#pragma unroll
    for (int c = 0; c < TW; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = i0 + wr + 16 * a + (l >> 4) + 4 * r, j = j0 + wc + 16 * c + (l & 15);
        if (i < M && j < N && i <= j) {
          gbl_t<double>* p = C + (k0 + i) + (size_t)(k0 + j) * ld;
          *p = *p - acc[a][c][r];
        }
      }
}

struct PrepArgs {
  int batch, n_max, k0, nb;
  const int* n_in;       // the caller's orders
  const int* ld;
  double* const* x;
  int* n_use;            // order in use: the caller's, 0 once invalid
  int* n_blk;            // diagonal block order at this panel
  int* m_rhs;            // columns right of the diagonal block
  double** diag;         // diagonal block
  double** panel;        // block right of it
  int* info;             // the caller's info (validation at the first panel)
  tla_stat* stat;
};

__global__ void k_panel_prep(PrepArgs g) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= g.batch) return;
  int n;
  if (g.k0 == 0) {
    n = g.n_in[b];
    int st = 0;
    if (n < 0 || n > g.n_max) st = -1;
    else if (g.ld[b] < (n > 1 ? n : 1)) st = -2;
    g.info[b] = st;
    if (st != 0) n = 0;
    g.n_use[b] = n;
    if (g.stat) {
      g.stat[b].iters = 0;
      g.stat[b].flags = 0;
      g.stat[b].eta = 0.0;
    }
  } else {
    n = g.n_use[b];
  }
  const int rem = n - g.k0;
  const int nb = rem <= 0 ? 0 : (rem < g.nb ? rem : g.nb);
  g.n_blk[b] = nb;
  g.m_rhs[b] = rem > g.nb ? rem - g.nb : 0;
  const int ld = g.ld[b];
  double* x = g.x[b];
  // pointers stay inside the matrix where nothing is left to do
  const int k = nb > 0 ? g.k0 : 0;
  g.diag[b] = x + k + (size_t)k * ld;
  g.panel[b] = x + k + (size_t)(nb > 0 && rem > g.nb ? g.k0 + g.nb : k) * ld;
}

// The first failing pivot of this panel's diagonal block, as a leading minor
// of the whole matrix; later panels of a failed instance are skipped.
__global__ void k_panel_merge(int batch, int k0, const int* blk_info, int* info, int* n_use) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= batch) return;
  const int s = blk_info[b];
  if (info[b] == 0 && s > 0) {
    info[b] = k0 + s;
    n_use[b] = 0;
  }
}

// Panel solve B := X_kk^{-T} B, B the block right of the diagonal block.
// One workgroup of 12 waves per (instance, 12 column tiles of B): the
// block's upper triangle is staged in LDS once (zero below the diagonal, one
// on the padded diagonal), and each wave solves one 16-column tile of B held
// in registers, tile row by tile row.  The FP64 accumulator layout of the
// matrix cores (lane l: column l & 15, rows (l >> 4) + 4r) is also the layout
// of their B operand for the four k-steps of a 16-deep product, so the solved
// tiles feed the products X_KI^T Z_K directly from registers.
// 12 waves: three per SIMD leave each wave the registers for its eight
// solution tiles (16 waves spilled); scratch: the strip solver's 16 x 17 tile
constexpr int kTsNW = 12, kTsNT = kPanelNB / 16, kTsLd = 17, kTsTile = 16 * kTsLd, kTsScr = kTsTile;

struct SolveArgs {
  const int* n_blk;
  const int* m_rhs;
  const int* ld;
  double* const* diag;
  double* const* panel;
};

TLA_DI int tri_index(int k, int i) { return i * (i + 1) / 2 + k; }  // upper tile (k, i), k <= i

__global__ __launch_bounds__(kTsNW * 64) void k_panel_trsm(SolveArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  const int n = g.n_blk[b], m = g.m_rhs[b];
  if (n <= 0 || m <= 0 || blockIdx.y * kTsNW * 16 >= m) return;
  const int ld = g.ld[b];
  const gbl_t<double>* X = to_gbl(static_cast<const double*>(g.diag[b]));
  lds_t<double>* S = to_lds(reinterpret_cast<double*>(smem));
  lds_t<double>* wbuf = S + kTsNT * (kTsNT + 1) / 2 * kTsTile + wave_id() * kTsScr;
  const int nt = (n + 15) / 16;
  // stage the upper tiles, column-major inside each tile (coalesced along rows)
  const int ntile = nt * (nt + 1) / 2;
  for (int q = threadIdx.x; q < ntile * 256; q += blockDim.x) {
    const int tix = q >> 8, e = q & 255, r = e & 15, c = e >> 4;
    int i = 0;
    while ((i + 1) * (i + 2) / 2 <= tix) ++i;
    const int k = tix - i * (i + 1) / 2;
    const int row = 16 * k + r, col = 16 * i + c;
    const int rr = row < n ? row : n - 1, cc = col < n ? col : n - 1;
    const double raw = X[rr + (size_t)cc * ld];
    double v;
    if (row < n && col < n) v = row <= col ? raw : 0.0;
    else v = row == col ? 1.0 : 0.0;
    S[tix * kTsTile + r + c * kTsLd] = v;
  }
  __syncthreads();
  const int J = blockIdx.y * kTsNW + wave_id();
  if (16 * J >= m) return;
  const int l = lane_id(), jc = 16 * J + (l & 15), kq = l >> 4;
  gbl_t<double>* B = to_gbl(g.panel[b]);
  const bool cin = jc < m;
  const int jcc = cin ? jc : m - 1;
  Tile<double, 16> Z[kTsNT];
#pragma unroll
  for (int I = 0; I < kTsNT; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * I + kq + 4 * r;
      const int rr = row < n ? row : n - 1;
      const double raw = B[rr + (size_t)jcc * ld];
      Z[I].v[r] = (row < n && cin) ? raw : 0.0;
    }
#pragma unroll
  for (int I = 0; I < kTsNT; ++I) {
    if (I >= nt) break;
    d4 acc = {Z[I].v[0], Z[I].v[1], Z[I].v[2], Z[I].v[3]};
#pragma unroll
    for (int K = 0; K < I; ++K) {
      const lds_t<double>* T = S + tri_index(K, I) * kTsTile;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-T[(4 * kk + kq) + (l & 15) * kTsLd], Z[K].v[kk], acc, 0, 0, 0);
    }
    Tile<double, 16> c;
#pragma unroll
    for (int r = 0; r < 4; ++r) c.v[r] = acc[r];
    tile_trsm_ut<double, 16>(c, View<double, true>{S + tri_index(I, I) * kTsTile, 1, kTsLd}, wbuf);
    Z[I] = c;
  }
#pragma unroll
  for (int I = 0; I < kTsNT; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * I + kq + 4 * r;
      if (row < n && cin) B[row + (size_t)jc * ld] = Z[I].v[r];
    }
}

size_t panel_trsm_lds() { return ((size_t)kTsNT * (kTsNT + 1) / 2 * kTsTile + (size_t)kTsNW * kTsScr) * sizeof(double); }

// ======================================================= Sylvester by blocks
// L X + X U = C for the large sizes as a wavefront over NB x NB blocks (NB = 128): the
// blocks (I, J) with I + J = d are independent once the earlier anti-diagonals
// are solved, and each needs
//   C_IJ -= L_{I,<I} X_{<I,J} + X_{I,<J} U_{<J,J}     (update)
//   L_II X_IJ + X_IJ U_JJ = C_IJ                        (block solve)
// Each anti-diagonal is two launches over the whole batch: the updates as
// batched FP64 matrix-core products (two k-loops into one accumulator), then
// the block solves, one workgroup per block, by the tile wavefront of the
// in-place kernels on rectangular blocks (the last block row and column are
// shorter when NB does not divide n).

struct SylArgs {
  int batch, nb, d;
  const int* n;          // order in use (0: skip the instance)
  const double* const* l;
  const int* ldl;
  const double* const* u;
  const int* ldu;
  double* const* c;
  const int* ldc;
};

// grid (1, block row I, instance): the update of block (I, d - I), NB = 128
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_bgemm_syl(SylArgs g) {
  constexpr int BM = 128, TW = Core<BM>::TW;
  __shared__ double sA[kBk * Core<BM>::LD];
  __shared__ double sB[kBk * Core<BM>::LD];
  const int b = blockIdx.z, I = blockIdx.y, J = g.d - I;
  const int n = g.n[b], nb = g.nb;
  const int P = (n + nb - 1) / nb;
  if (J < 0 || I >= P || J >= P) return;
  const int mI = n - I * nb < nb ? n - I * nb : nb, nJ = n - J * nb < nb ? n - J * nb : nb;
  const int ldl = g.ldl[b], ldu = g.ldu[b], ldc = g.ldc[b];
  const gbl_t<double>* L = to_gbl(g.l[b]);
  const gbl_t<double>* U = to_gbl(g.u[b]);
  gbl_t<double>* X = to_gbl(g.c[b]);
  const int rI = I * nb, cJ = J * nb;
  d4v acc[TW][TW];
  zero_acc<TW>(acc);
  // L_{I,<I} X_{<I,J}, then X_{I,<J} U_{<J,J} (one copy of the core: a
  // loop, not two inlined calls, keeps the registers within budget)
#pragma unroll 1
  for (int pass = 0; pass < 2; ++pass) {
    const gbl_t<double>* A = pass == 0 ? L + rI : X + rI;
    const gbl_t<double>* B = pass == 0 ? X + (size_t)cJ * ldc : U + (size_t)cJ * ldu;
    bgemm_core<BM, false>(acc, A, pass == 0 ? ldl : ldc, B, pass == 0 ? ldc : ldu, (pass == 0 ? I : J) * nb, mI,
                          nJ, to_lds(sA), to_lds(sB));
  }
  const int l = lane_id(), w = wave_id(), wr = (w >> 1) * (BM / 2), wc = (w & 1) * (BM / 2);
#pragma unroll
  for (int a = 0; a < TW; ++a)
#pragma unroll
    for (int c = 0; c < TW; ++c)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = wr + 16 * a + (l >> 4) + 4 * r, j = wc + 16 * c + (l & 15);
        if (i < mI && j < nJ) {
          gbl_t<double>* p = X + (rI + i) + (size_t)(cJ + j) * ldc;
          *p = *p - acc[a][c][r];
        }
      }
}

// In/out view of an nr x nc block of a column-major matrix: reads outside
// return 0, writes there are dropped.
struct BlockIO {
  double* p;
  int ld, nr, nc, r0, c0;
  TLA_DI double operator()(int i, int j) const {
    const int r = r0 + i, c = c0 + j;
    const int rr = r < nr ? r : nr - 1, cc = c < nc ? c : nc - 1;
    const double raw = to_gbl(p)[rr + (size_t)cc * ld];
    return (r < nr && c < nc) ? raw : 0.0;
  }
  TLA_DI void store(int i, int j, double v) const {
    const int r = r0 + i, c = c0 + j;
    if (r < nr && c < nc) to_gbl(p)[r + (size_t)c * ld] = v;
  }
  TLA_DI void fence() const { __threadfence_block(); }
  TLA_DI BlockIO sub(int i0, int j0) const {
    BlockIO v = *this;
    v.r0 += i0;
    v.c0 += j0;
    return v;
  }
};

constexpr int kSbNW = 4;    // (8 waves measured slower)
constexpr int kSylNB = 128;  // block order (one 128 x 128 update block)

// grid (block row I, instance): the block (I, d - I) by the tile wavefront
__global__ __launch_bounds__(kSbNW * 64) void k_syl_blocks(SylArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.y, I = blockIdx.x, J = g.d - I;
  const int n = g.n[b], nb = g.nb;
  const int P = (n + nb - 1) / nb;
  if (J < 0 || I >= P || J >= P) return;
  const int mI = n - I * nb < nb ? n - I * nb : nb, nJ = n - J * nb < nb ? n - J * nb : nb;
  const int ldl = g.ldl[b], ldu = g.ldu[b], ldc = g.ldc[b];
  const GView<double> Lb = gview<double>(g.l[b] + (size_t)I * nb * (1 + (size_t)ldl), ldl, mI, -1);
  const GView<double> Ub = gview<double>(g.u[b] + (size_t)J * nb * (1 + (size_t)ldu), ldu, nJ, +1);
  const BlockIO X{g.c[b] + (size_t)I * nb + (size_t)J * nb * ldc, ldc, mI, nJ, 0, 0};
  lds_t<double>* wbuf = to_lds(reinterpret_cast<double*>(smem) + wave_id() * wave_scratch(16));
  typedef Gemm<double, 16, ENG_MFMA> G;
  const int ntr = (mI + 15) / 16, ntc = (nJ + 15) / 16, w = wave_id();
  for (int dd = 0; dd <= ntr + ntc - 2; ++dd) {
    const int lo = dd - ntc + 1 > 0 ? dd - ntc + 1 : 0, hi = dd < ntr - 1 ? dd : ntr - 1;
    for (int Ii = lo + w; Ii <= hi; Ii += kSbNW) {
      const int Jj = dd - Ii;
      const auto k = sylv_fetch<double, 16>(Lb.sub(16 * Ii, 16 * Ii), Ub.sub(16 * Jj, 16 * Jj));
      Tile<double, 16> c;
      tload(c, X.sub(16 * Ii, 16 * Jj));
      gemm_sum<G>(c, 0, Ii, [&](int K) { return Lb.sub(16 * Ii, 16 * K); }, [&](int K) { return X.sub(16 * K, 16 * Jj); });
      gemm_sum<G>(c, 0, Jj, [&](int K) { return X.sub(16 * Ii, 16 * K); }, [&](int K) { return Ub.sub(16 * K, 16 * Jj); });
      sylv_solve<double, 16>(c, k, wbuf, mI - 16 * Ii, nJ - 16 * Jj);
      tstore(c, X.sub(16 * Ii, 16 * Jj));
    }
    __syncthreads();
  }
}

// per instance: argument checks, the first zero denominator l_ii + u_jj
// (column-major order, as the in-place kernels report it), refinement record
struct SylPrep {
  int n_max;
  const int* n_in;
  const double* const* l;
  const int* ldl;
  const double* const* u;
  const int* ldu;
  const int* ldc;
  int* n_use;
  int* info;
  tla_stat* stat;
};

__global__ __launch_bounds__(256) void k_syl_prep(SylPrep g) {
  __shared__ int s_info;
  const int b = blockIdx.x;
  const int n = g.n_in[b];
  int st = 0;
  if (n < 0 || n > g.n_max) st = -1;
  else if (g.ldl[b] < (n > 1 ? n : 1) || g.ldu[b] < (n > 1 ? n : 1) || g.ldc[b] < (n > 1 ? n : 1)) st = -2;
  if (threadIdx.x == 0) s_info = INT_MAX;
  __syncthreads();
  if (st == 0 && n > 0)
    scan_zero_denoms(gview<double>(g.l[b], g.ldl[b], n, -1), gview<double>(g.u[b], g.ldu[b], n, +1), n, false,
                     &s_info);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (st == 0 && s_info != INT_MAX) st = s_info;
    g.info[b] = st;
    g.n_use[b] = st == 0 ? n : 0;
    if (g.stat) {
      g.stat[b].iters = 0;
      g.stat[b].flags = 0;
      g.stat[b].eta = 0.0;
    }
  }
}

}  // namespace

// Large FP64 Sylvester by the block wavefront; a as for the in-place kernels.
tla_status trsyl_blocks(tla_ctx* h, const KArgs& a) {
  const int batch = a.batch, nb = kSylNB;
  const size_t bytes = (size_t)batch * sizeof(int);
  if (bytes > h->panel_bytes) {
    if (h->panel_work) {
      PN_HIP(hipStreamSynchronize(h->stream));
      hipFree(h->panel_work);
      h->panel_work = nullptr;
      h->panel_bytes = 0;
    }
    if (hipMalloc(&h->panel_work, bytes) != hipSuccess) return TLA_E_NOMEM;
    h->panel_bytes = bytes;
  }
  int* n_use = reinterpret_cast<int*>(h->panel_work);
  SylPrep sp{a.n_max, a.n, a.a, a.lda, a.b, a.ldb, a.ldc, n_use, a.info, a.stat};
  hipLaunchKernelGGL(k_syl_prep, dim3(batch), dim3(256), 0, h->stream, sp);
  PN_HIP(hipGetLastError());
  const int P = (a.n_max + nb - 1) / nb;
  const size_t lds = (size_t)kSbNW * wave_scratch(16) * sizeof(double);
  for (int d = 0; d <= 2 * P - 2; ++d) {
    SylArgs ga{batch, nb, d, n_use, a.a, a.lda, a.b, a.ldb, a.c, a.ldc};
    if (d > 0) {
      hipLaunchKernelGGL(k_bgemm_syl, dim3(1, P, batch), dim3(256), 0, h->stream, ga);
      PN_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_syl_blocks, dim3(P, batch), dim3(64 * kSbNW), lds, h->stream, ga);
    PN_HIP(hipGetLastError());
  }
  return TLA_OK;
}

// Large FP64 Cholesky by block panels; a as for the in-place kernels.
tla_status potrf_panel(tla_ctx* h, const KArgs& a) {
  const int batch = a.batch;
  // workspace: four int arrays and two pointer arrays
  const size_t ints = (size_t)4 * batch * sizeof(int);
  const size_t ptr_off = (ints + 255) & ~(size_t)255;
  const size_t bytes = ptr_off + (size_t)2 * batch * sizeof(double*);
  if (bytes > h->panel_bytes) {
    if (h->panel_work) {
      PN_HIP(hipStreamSynchronize(h->stream));
      hipFree(h->panel_work);
      h->panel_work = nullptr;
      h->panel_bytes = 0;
    }
    if (hipMalloc(&h->panel_work, bytes) != hipSuccess) return TLA_E_NOMEM;
    h->panel_bytes = bytes;
  }
  char* base = reinterpret_cast<char*>(h->panel_work);
  int* n_use = reinterpret_cast<int*>(base);
  int* n_blk = n_use + batch;
  int* m_rhs = n_use + 2 * batch;
  int* blk_info = n_use + 3 * batch;
  double** diag = reinterpret_cast<double**>(base + ptr_off);
  double** panel = reinterpret_cast<double**>(diag + batch);

  const int nb = kPanelNB;
  // diagonal blocks: in place, four waves per block (the batch is small
  // next to the number of compute units)
  tla_plan pd = default_plan(TLA_POTRF, nb, TLA_F64);
  pd.variant = 1;  // left-looking: a block row's tiles go to all four waves
  pd.waves = 4;
  const dim3 pg((batch + 255) / 256), pb(256);
  for (int k0 = 0; k0 < a.n_max; k0 += nb) {
    if (k0 > 0) {
      PanelArgs ga{batch, a.n_max, k0, nb, n_use, a.c, a.ldc};
      const dim3 grid((a.n_max - k0 + kCholBM - 1) / kCholBM, (nb + kCholBM - 1) / kCholBM, batch);
      hipLaunchKernelGGL(k_bgemm_chol, grid, dim3(256), 0, h->stream, ga);
      PN_HIP(hipGetLastError());
    }
    PrepArgs pa{batch, a.n_max, k0, nb, a.n, a.ldc, a.c, n_use, n_blk, m_rhs, diag, panel, a.info, a.stat};
    hipLaunchKernelGGL(k_panel_prep, pg, pb, 0, h->stream, pa);
    PN_HIP(hipGetLastError());
    // diagonal block
    KArgs kd{};
    kd.batch = batch;
    kd.n_max = nb;
    kd.n = n_blk;
    kd.c = diag;
    kd.ldc = a.ldc;
    kd.info = blk_info;
    tla_status s = launch(h, TLA_POTRF, TLA_F64, pd, kd);
    if (s != TLA_OK) return s;
    // panel solve with the block's factor (skipped where the block failed:
    // its instance is then unspecified, as the caller's contract allows)
    if (k0 + nb < a.n_max) {
      SolveArgs sa{n_blk, m_rhs, a.ldc, diag, panel};
      const size_t lds = panel_trsm_lds();
      PN_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_panel_trsm),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
      const int tiles = (a.n_max - k0 - nb + 15) / 16;
      hipLaunchKernelGGL(k_panel_trsm, dim3(batch, (tiles + kTsNW - 1) / kTsNW), dim3(64 * kTsNW), lds, h->stream,
                         sa);
      PN_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_panel_merge, pg, pb, 0, h->stream, batch, k0, blk_info, a.info, n_use);
    PN_HIP(hipGetLastError());
  }
  return TLA_OK;
}

}  // namespace tla
