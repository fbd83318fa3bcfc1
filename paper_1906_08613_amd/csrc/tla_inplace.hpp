// In-place solver bodies: the matrices stay in global memory and are solved
// in place; only the tile solvers' scratch lives in LDS.  Tiles stream through
// registers and the matrix cores (16 x 16 tiles), the same blocked variants as
// for the LDS-resident kernels.  Used for the large sizes (n > 128, one
// workgroup of 16 wavefronts per instance), as placement 3 of the smaller
// sizes (1, 2 or 4 wavefronts: with no matrix in LDS many more instances are
// resident per compute unit, and the caches serve the tile traffic) and by
// the ragged workers.
#pragma once
#include "tla_kernels.hpp"

namespace tla {

// In/out view of the caller's matrix for in-place solves.  Reads outside
// n x n return the padding (1 on the diagonal for the Cholesky pivots, 0
// elsewhere) and writes there are dropped.  upper_only (Cholesky): the strict
// lower triangle is neither read (reads return 0) nor written.  SYM
// (Lyapunov): the matrix is symmetric and held by its lower triangle, so a
// read above the diagonal returns the mirrored element, and mirrors() tells
// the tile solvers to store every solved tile below the diagonal also
// transposed above it.
template <class T, bool SYM = false, class S = double>
struct IOView {
  S* p;  // storage type of the caller's matrix (FP64, or FP32 for the FP32-I/O entry points)
  int ld, n;
  bool upper_only;
  int r0, c0;
  bool tr;
  TLA_DI void coords(int i, int j, int& r, int& c) const {
    r = tr ? r0 + j : r0 + i;
    c = tr ? c0 + i : c0 + j;
  }
  TLA_DI T operator()(int i, int j) const {
    int r, c;
    coords(i, j, r, c);
    if constexpr (SYM) {
      if (r < c) { const int t = r; r = c; c = t; }
    }
    const bool in = r < n && c < n;
    const int rr = r < n ? r : n - 1, cc = c < n ? c : n - 1;
    const S raw = to_gbl(p)[rr + (size_t)cc * ld];
    if (!in) return (upper_only && r == c) ? T(1) : T(0);
    return (upper_only && r > c) ? T(0) : T(raw);
  }
  TLA_DI void store(int i, int j, T v) const {
    int r, c;
    coords(i, j, r, c);
    if (r < n && c < n && !(upper_only && r > c)) to_gbl(p)[r + (size_t)c * ld] = S(v);
  }
  // the 16 x 16 block at (r0, c0) lies inside n x n and strictly above the
  // diagonal where only the upper triangle is read, so raw() may read it
  // without clamping or selects.  Used by the Cholesky products (both
  // operands are views of the factor); for the symmetric Lyapunov view the
  // unmasked path measured slower and stays compiled out.
  TLA_DI bool interior16() const {
    if constexpr (SYM) return false;
    const int rhi = r0 + 15, chi = c0 + 15;
    if (rhi >= n || chi >= n) return false;
    if (upper_only && rhi > c0) return false;
    return true;
  }
  TLA_DI T raw(int i, int j) const {
    int r, c;
    coords(i, j, r, c);
    return T(to_gbl(p)[r + (size_t)c * ld]);
  }
  TLA_DI void fence() const { __threadfence_block(); }
  static constexpr bool mirrors() { return SYM; }
  TLA_DI IOView sub(int i0, int j0) const {
    IOView v = *this;
    if (tr) { v.r0 += j0; v.c0 += i0; } else { v.r0 += i0; v.c0 += j0; }
    return v;
  }
  TLA_DI IOView t() const { IOView v = *this; v.tr = !tr; return v; }
};

template <class T, class S>
TLA_DI IOView<T, false, S> ioview(S* p, int ld, int n, bool upper_only) {
  return IOView<T, false, S>{p, ld, n, upper_only, 0, 0, false};
}

constexpr int kLargeTB = 16, kLargeNW = 16;


// T is the element type of both the arithmetic and the caller's matrices:
// double for the FP64 entry points, float for the FP32-I/O ones (the
// instance's pointers are then float arrays; KArgs carries them untyped).
template <int NW, class T = double>
TLA_DI void large_ctx_init(unsigned char* smem, Ctx<T>& cx, int n, int*& s_info, int init) {
  T* wb = reinterpret_cast<T*>(smem);
  s_info = reinterpret_cast<int*>(wb + NW * wave_scratch(kLargeTB));
  if (threadIdx.x == 0) *s_info = init;
  __syncthreads();
  cx = Ctx<T>{n, (n + kLargeTB - 1) / kLargeTB, to_lds(wb + wave_id() * wave_scratch(kLargeTB)), to_lds(s_info)};
}

template <class T>
TLA_DI T* as_elem(double* p) { return reinterpret_cast<T*>(p); }
template <class T>
TLA_DI const T* as_elem(const double* p) { return reinterpret_cast<const T*>(p); }

template <int NW, int VAR, class T = double>
TLA_DI void potrf_inplace_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  int n;
  if (skip_unflagged(g, in)) return;
  if (!validate(in, g.n_max, n)) return;
  Ctx<T> cx;
  int* s_info;
  large_ctx_init<NW, T>(smem, cx, n, s_info, 0);
  potrf_blocked<T, kLargeTB, ENG_MFMA, NW, VAR>(ioview<T>(as_elem<T>(in.c), in.ldc, n, true), cx);
  __syncthreads();
  if (threadIdx.x == 0) {
    *in.info = *s_info;
    if (in.stat && !g.only_flagged) { in.stat->iters = 0; in.stat->flags = 0; in.stat->eta = 0.0; }
  }
}

template <int NW, int VAR, class T = double>
TLA_DI void trsyl_inplace_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  int n;
  if (skip_unflagged(g, in)) return;
  if (!validate(in, g.n_max, n)) return;
  Ctx<T> cx;
  int* s_info;
  large_ctx_init<NW, T>(smem, cx, n, s_info, INT_MAX);
  const auto L = gview<T>(as_elem<T>(in.a), in.lda, n, -1);
  const auto U = gview<T>(as_elem<T>(in.b), in.ldb, n, +1);
  scan_zero_denoms(L, U, n, false, s_info);
  trsyl_blocked<T, kLargeTB, ENG_MFMA, NW, VAR>(ioview<T>(as_elem<T>(in.c), in.ldc, n, false), L, U, cx);
  __syncthreads();
  if (threadIdx.x == 0) {
    *in.info = *s_info == INT_MAX ? 0 : *s_info;
    if (in.stat && !g.only_flagged) { in.stat->iters = 0; in.stat->flags = 0; in.stat->eta = 0.0; }
  }
}

template <int NW, int VAR, class T = double>
TLA_DI void trlyap_inplace_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  int n;
  if (skip_unflagged(g, in)) return;
  if (!validate(in, g.n_max, n)) return;
  Ctx<T> cx;
  int* s_info;
  large_ctx_init<NW, T>(smem, cx, n, s_info, INT_MAX);
  const auto L = gview<T>(as_elem<T>(in.a), in.lda, n, -1);
  scan_zero_denoms(L, L, n, true, s_info);
  // S is given by its lower triangle: the view reads the diagonal tiles'
  // upper halves from it, and the solved tiles are stored on both sides
  const IOView<T, true, T> X{as_elem<T>(in.c), in.ldc, n, false, 0, 0, false};
  trlyap_blocked<T, kLargeTB, ENG_MFMA, NW, VAR>(X, L, cx);
  __syncthreads();
  if (threadIdx.x == 0) {
    *in.info = *s_info == INT_MAX ? 0 : *s_info;
    if (in.stat && !g.only_flagged) { in.stat->iters = 0; in.stat->flags = 0; in.stat->eta = 0.0; }
  }
}

}  // namespace tla
