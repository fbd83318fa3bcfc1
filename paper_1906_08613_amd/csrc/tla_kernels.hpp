// Batched kernels: one workgroup per instance, operands staged in LDS.
//
// Every kernel reads the instance's n and leading dimensions from device
// arrays, validates them (info = -1 / -2 and skip), loads the referenced
// triangles with column-coalesced loads into LDS, runs one blocked variant
// and writes the referenced part of the result back in place.
#pragma once
#ifdef __HIPCC_RTC__
// (compiled at run time by the exact-size path: no C library headers there)
#ifndef INT_MAX
#define INT_MAX __INT_MAX__
#endif
#else
#include <climits>
#endif

#include "tla_solvers.hpp"
#include "tla_internal.h"

namespace tla {

// ----------------------------------------------------------- global views
// Read-only view of a caller matrix in global memory, with the coordinates
// of the underlying column-major matrix.  Entries outside n x n or outside
// the referenced triangle (tri -1: lower, +1: upper) read as zero, so padded
// tiles need no special casing; tri +2 / -2 read a symmetric matrix from its
// upper / lower triangle.
template <class T, class S = double>
struct GView {
  const S* p;  // storage type of the caller's matrix (FP64, or FP32 for the FP32-I/O entry points)
  int ld, n, tri;
  int r0, c0;
  bool tr;
  TLA_DI T operator()(int i, int j) const {
    const int r = tr ? r0 + j : r0 + i;
    const int c = tr ? c0 + i : c0 + j;
    const bool in = r < n && c < n;
    int rr = r < n ? r : n - 1, cc = c < n ? c : n - 1;
    if (tri == 2 || tri == -2) {  // symmetric, stored in the upper (2) or lower (-2) triangle
      const bool swap = tri == 2 ? rr > cc : rr < cc;
      if (swap) { const int t = rr; rr = cc; cc = t; }
    }
    // unconditional load from a clamped address, then select
    const S raw = to_gbl(p)[rr + (size_t)cc * ld];
    const bool ok = in && (tri == 0 || tri == 2 || tri == -2 || (tri < 0 ? r >= c : r <= c));
    return ok ? T(raw) : T(0);
  }
  TLA_DI GView sub(int i0, int j0) const {
    GView v = *this;
    if (tr) { v.r0 += j0; v.c0 += i0; } else { v.r0 += i0; v.c0 += j0; }
    return v;
  }
  TLA_DI GView t() const { GView v = *this; v.tr = !tr; return v; }
};
template <class T, class S>
TLA_DI GView<T, S> gview(const S* p, int ld, int n, int tri) { return GView<T, S>{p, ld, n, tri, 0, 0, false}; }

// ------------------------------------------------------ ingest / egress
// Copies the n x n global matrix into the np x np work matrix (ld = ldw; in
// LDS, or in global memory for !LDS),
// keeping the part selected by `part` and writing `pad` on the padded
// diagonal and zero elsewhere.  part: 0 full, -1 lower (i >= j), +1 upper.
// Rows go to lanes (coalesced column reads), columns to waves; U columns are
// loaded before any is stored so that their latencies overlap.  Returns this
// thread's share of the squared Frobenius norm of the kept part, counting
// off-diagonal entries twice when `sym` (a symmetric matrix given by one
// triangle).
template <class T, int NW, bool LDS = true>
TLA_DI double ingest(T* Wg, int ldw, int np, const double* Gg, int ldg, int n, int part, T pad, bool sym = false) {
  constexpr int U = 8;
  const int w = wave_id(), l = lane_id();
  const auto W = xcolmajor<!LDS>(Wg, ldw).p;
  const gbl_t<double>* G = to_gbl(Gg);
  double ss = 0.0;
  for (int i0 = 0; i0 < np; i0 += 64) {
    const int i = i0 + l;
    for (int jb = w; jb < np; jb += NW * U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        // unconditional load from a clamped address inside the kept part of
        // the column (so no cache line outside it is fetched), then select
        const int j = jb + u * NW;
        const int jc = j < n ? j : n - 1;
        int ic = i < n ? i : n - 1;
        if (part < 0) ic = ic > jc ? ic : jc;
        if (part > 0) ic = ic < jc ? ic : jc;
        const double raw = G[ic + (size_t)jc * ldg];
        const bool keep = i < n && j < n && (part == 0 || (part < 0 ? i >= j : i <= j));
        v[u] = keep ? raw : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = jb + u * NW;
        if (i < np && j < np) {
          const bool inside = i < n && j < n;
          W[i + j * ldw] = inside ? T(v[u]) : (i == j ? pad : T(0));
          ss += (sym && i != j ? 2.0 : 1.0) * v[u] * v[u];
        }
      }
    }
  }
  return ss;
}

// Mirrors the lower triangle of an np x np LDS matrix into its upper triangle
// (call between barriers).
template <class T, bool LDS = true>
TLA_DI void mirror_lower(T* Wg, int ldw, int np) {
  const View<T, LDS> Wv = xcolmajor<!LDS>(Wg, ldw);
  auto* W = Wv.p;
  for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
    const int j = e / np, i = e - j * np;
    if (i < j) W[i + j * ldw] = W[j + i * ldw];
  }
}

// Writes the n x n result back: part 0 full, +1 upper triangle only,
// 2 symmetric from the lower triangle.  The source is in LDS unless !LDS.
template <class T, int NW, bool LDS = true>
TLA_DI void egress(double* Gg, int ldg, int n, const T* Wg, int ldw, int part) {
  const int w = wave_id(), l = lane_id();
  const View<T, LDS> Wv = xcolmajor<!LDS>(const_cast<T*>(Wg), ldw);
  const auto* W = Wv.p;
  gbl_t<double>* G = to_gbl(Gg);
  for (int j = w; j < n; j += NW) {
    for (int i = l; i < n; i += 64) {
      if (part == 1 && i > j) continue;
      const T v = (part == 2 && i < j) ? W[j + i * ldw] : W[i + j * ldw];
      G[i + (size_t)j * ldg] = double(v);
    }
  }
}

// value of v held by lane l of this wavefront (l uniform across the wave)
TLA_DI double read_lane(double v, int l) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

// First zero denominator d_ij = a_ii + b_jj (column-major index i + j n, plus
// 1) into *info; lower_only restricts the scan to i >= j.  With F32 the same
// pass also reports (return value) whether some denominator is zero once the
// two diagonal entries are rounded to FP32 and added in FP32.  The (i, j)
// plane is cut into 64 x 64 chunks handed to the waves; a wave loads the two
// diagonal pieces of its chunk once, one element per lane, and walks the
// columns with b_jj broadcast from lane j.  Each thread keeps its own minimum
// and publishes it once.
template <bool F32 = false, class VA, class VB, class IP>
TLA_DI bool scan_zero_denoms(const VA& A, const VB& B, int n, bool lower_only, IP info) {
  int best = INT_MAX;
  bool zero32 = false;
  const int nw = blockDim.x >> 6, lane = lane_id();
  const int nc = (n + 63) >> 6;
  for (int t = wave_id(); t < nc * nc; t += nw) {
    const int ic = t % nc, jc = t / nc;
    if (lower_only && ic < jc) continue;
    const int i = 64 * ic + lane, jl = 64 * jc + lane;
    const int ii = i < n ? i : n - 1, jj = jl < n ? jl : n - 1;
    const double ai = A(ii, ii);
    const double bl = B(jj, jj);
    const float ai32 = float(ai);
    const int jn = n - 64 * jc < 64 ? n - 64 * jc : 64;
    for (int q = 0; q < jn; ++q) {
      const double bj = read_lane(bl, q);
      const int j = 64 * jc + q;
      const bool live = i < n && (!lower_only || i >= j);
      if (live && ai + bj == 0.0) best = min(best, 1 + i + j * n);
      if constexpr (F32) zero32 = zero32 || (live && ai32 + float(bj) == 0.0f);
    }
  }
  if (best != INT_MAX) atomicMin(info, best);
  return zero32;
}

// Squared Frobenius norm share of this thread for the part of an n x n
// global matrix selected by `part` (0 full, -1 lower, +1 upper); sym counts
// off-diagonal entries twice.  Loads are batched as in ingest.
template <int NW>
TLA_DI double gnorm2(const double* Gg, int ldg, int n, int part, bool sym = false) {
  constexpr int U = 8;
  const int w = wave_id(), l = lane_id();
  const gbl_t<double>* G = to_gbl(Gg);
  double ss = 0.0;
  for (int i0 = 0; i0 < n; i0 += 64) {
    const int i = i0 + l;
    for (int jb = w; jb < n; jb += NW * U) {
      double v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = jb + u * NW;
        const int jc = j < n ? j : n - 1;
        int ic = i < n ? i : n - 1;
        if (part < 0) ic = ic > jc ? ic : jc;
        if (part > 0) ic = ic < jc ? ic : jc;
        const double raw = G[ic + (size_t)jc * ldg];
        const bool keep = i < n && j < n && (part == 0 || (part < 0 ? i >= j : i <= j));
        v[u] = keep ? raw : 0.0;
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int j = jb + u * NW;
        ss += (sym && i != j ? 2.0 : 1.0) * v[u] * v[u];
      }
    }
  }
  return ss;
}

// One instance's operands and result slots (see KArgs for the roles).
struct Inst {
  int n;
  const double* a;
  int lda;
  const double* b;
  int ldb;
  double* c;
  int ldc;
  int* info;
  tla_stat* stat;
};

TLA_DI Inst fetch_uniform(const KArgs& g, int b) {
  Inst in;
  in.n = g.n[b];
  in.a = g.a ? g.a[b] : nullptr;
  in.lda = g.lda ? g.lda[b] : 1;
  in.b = g.b ? g.b[b] : nullptr;
  in.ldb = g.ldb ? g.ldb[b] : 1;
  in.c = g.c[b];
  in.ldc = g.ldc[b];
  in.info = g.info + b;
  in.stat = g.stat ? g.stat + b : nullptr;
  return in;
}

// Checks n and the leading dimensions of the matrices the instance uses;
// writes info = -1 / -2 (or 0 for n = 0) and returns false to skip it.
TLA_DI bool validate(const Inst& in, int n_max, int& n) {
  n = in.n;
  int bad = 0;
  if (n < 0 || n > n_max) bad = -1;
  else {
    const int m = n > 1 ? n : 1;
    if (in.ldc < m) bad = -2;
    if (in.a && in.lda < m) bad = -2;
    if (in.b && in.ldb < m) bad = -2;
  }
  if (bad != 0 || n == 0) {
    if (threadIdx.x == 0) {
      *in.info = bad;
      if (in.stat) { in.stat->iters = 0; in.stat->flags = 0; in.stat->eta = 0.0; }
    }
    return false;
  }
  return true;
}

// Second (FP64) pass after a mixed launch whose FP64 solution did not fit in
// LDS: only instances that the mixed kernel left unconverged are solved.
TLA_DI bool skip_unflagged(const KArgs& g, const Inst& in) {
  if (!g.only_flagged) return false;
  if (in.n <= 0 || in.n > g.n_max || *in.info != 0) return true;
  return (in.stat->flags & TLA_STAT_CONVERGED) != 0;
}

// LDS bytes of the FP64 kernels for tile count ntmax per dimension.
__host__ __device__ inline size_t lds_mat_bytes(int ntmax, int tb, int elem) {
  const size_t np = (size_t)ntmax * tb;
  return np * (np + 1) * elem;
}
__host__ __device__ inline size_t lds_scratch_bytes(int nw, int tb, int elem) {
  return (size_t)nw * wave_scratch(tb) * elem + 16;
}

// ================================================================ FP64
template <int TB, int ENG, int NW, int VAR>
TLA_DI void potrf_f64_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  int n;
  if (skip_unflagged(g, in)) return;
  if (!validate(in, g.n_max, n)) return;
  const int nt = (n + TB - 1) / TB, np = nt * TB, ld = np + 1;
  double* A = reinterpret_cast<double*>(smem);
  double* wb = A + (size_t)g.ntmax * TB * (g.ntmax * TB + 1);
  int* s_info = reinterpret_cast<int*>(wb + NW * wave_scratch(TB));
  if (threadIdx.x == 0) *s_info = 0;
  ingest<double, NW>(A, ld, np, in.c, in.ldc, n, +1, 1.0);
  __syncthreads();
  Ctx<double> cx{n, nt, to_lds(wb + wave_id() * wave_scratch(TB)), to_lds(s_info)};
  potrf_blocked<double, TB, ENG, NW, VAR>(colmajor(A, ld), cx);
  __syncthreads();
  egress<double, NW>(in.c, in.ldc, n, A, ld, 1);
  if (threadIdx.x == 0) {
    *in.info = *s_info;
    if (in.stat && !g.only_flagged) { in.stat->iters = 0; in.stat->flags = 0; in.stat->eta = 0.0; }
  }
}

template <int TB, int ENG, int NW, int VAR>
__global__ __launch_bounds__(NW * 64) void k_potrf_f64(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  potrf_f64_body<TB, ENG, NW, VAR>(g, fetch_uniform(g, blockIdx.x), smem);
}

template <int TB, int ENG, int NW, int VAR, bool LU_LDS>
TLA_DI void trsyl_f64_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  int n;
  if (skip_unflagged(g, in)) return;
  if (!validate(in, g.n_max, n)) return;
  const int nt = (n + TB - 1) / TB, np = nt * TB, ld = np + 1;
  const size_t mat = (size_t)g.ntmax * TB * (g.ntmax * TB + 1);
  double* X = reinterpret_cast<double*>(smem);
  double* Ls = X + mat;
  double* Us = Ls + mat;
  double* wb = LU_LDS ? Us + mat : Ls;
  int* s_info = reinterpret_cast<int*>(wb + NW * wave_scratch(TB));
  if (threadIdx.x == 0) *s_info = INT_MAX;
  ingest<double, NW>(X, ld, np, in.c, in.ldc, n, 0, 0.0);
  if constexpr (LU_LDS) {
    ingest<double, NW>(Ls, ld, np, in.a, in.lda, n, -1, 0.0);
    ingest<double, NW>(Us, ld, np, in.b, in.ldb, n, +1, 0.0);
  }
  __syncthreads();
  Ctx<double> cx{n, nt, to_lds(wb + wave_id() * wave_scratch(TB)), to_lds(s_info)};
  if constexpr (LU_LDS) {
    scan_zero_denoms(colmajor(Ls, ld), colmajor(Us, ld), n, false, s_info);
    trsyl_blocked<double, TB, ENG, NW, VAR>(colmajor(X, ld), colmajor(Ls, ld), colmajor(Us, ld), cx);
  } else {
    const GView<double> L = gview<double>(in.a, in.lda, n, -1);
    const GView<double> U = gview<double>(in.b, in.ldb, n, +1);
    scan_zero_denoms(L, U, n, false, s_info);
    trsyl_blocked<double, TB, ENG, NW, VAR>(colmajor(X, ld), L, U, cx);
  }
  __syncthreads();
  egress<double, NW>(in.c, in.ldc, n, X, ld, 0);
  if (threadIdx.x == 0) {
    *in.info = *s_info == INT_MAX ? 0 : *s_info;
    if (in.stat && !g.only_flagged) { in.stat->iters = 0; in.stat->flags = 0; in.stat->eta = 0.0; }
  }
}

template <int TB, int ENG, int NW, int VAR, bool LU_LDS>
__global__ __launch_bounds__(NW * 64) void k_trsyl_f64(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  trsyl_f64_body<TB, ENG, NW, VAR, LU_LDS>(g, fetch_uniform(g, blockIdx.x), smem);
}

template <int TB, int ENG, int NW, int VAR, bool LU_LDS>
TLA_DI void trlyap_f64_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  int n;
  if (skip_unflagged(g, in)) return;
  if (!validate(in, g.n_max, n)) return;
  const int nt = (n + TB - 1) / TB, np = nt * TB, ld = np + 1;
  const size_t mat = (size_t)g.ntmax * TB * (g.ntmax * TB + 1);
  double* X = reinterpret_cast<double*>(smem);
  double* Ls = X + mat;
  double* wb = LU_LDS ? Ls + mat : Ls;
  int* s_info = reinterpret_cast<int*>(wb + NW * wave_scratch(TB));
  if (threadIdx.x == 0) *s_info = INT_MAX;
  ingest<double, NW>(X, ld, np, in.c, in.ldc, n, -1, 0.0);
  if constexpr (LU_LDS) ingest<double, NW>(Ls, ld, np, in.a, in.lda, n, -1, 0.0);
  __syncthreads();
  mirror_lower(X, ld, np);
  __syncthreads();
  Ctx<double> cx{n, nt, to_lds(wb + wave_id() * wave_scratch(TB)), to_lds(s_info)};
  if constexpr (LU_LDS) {
    scan_zero_denoms(colmajor(Ls, ld), colmajor(Ls, ld), n, true, s_info);
    trlyap_blocked<double, TB, ENG, NW, VAR>(colmajor(X, ld), colmajor(Ls, ld), cx);
  } else {
    const GView<double> L = gview<double>(in.a, in.lda, n, -1);
    scan_zero_denoms(L, L, n, true, s_info);
    trlyap_blocked<double, TB, ENG, NW, VAR>(colmajor(X, ld), L, cx);
  }
  __syncthreads();
  egress<double, NW>(in.c, in.ldc, n, X, ld, 2);
  if (threadIdx.x == 0) {
    *in.info = *s_info == INT_MAX ? 0 : *s_info;
    if (in.stat && !g.only_flagged) { in.stat->iters = 0; in.stat->flags = 0; in.stat->eta = 0.0; }
  }
}

template <int TB, int ENG, int NW, int VAR, bool LU_LDS>
__global__ __launch_bounds__(NW * 64) void k_trlyap_f64(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  trlyap_f64_body<TB, ENG, NW, VAR, LU_LDS>(g, fetch_uniform(g, blockIdx.x), smem);
}

}  // namespace tla
