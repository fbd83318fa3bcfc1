// Tile-level building blocks for the batched small solvers on CDNA4 (gfx950).
//
// One workgroup of NW wavefronts works on one problem instance whose operands
// sit in LDS (or, for the largest sizes, are read through the caches).  The
// matrix is cut into TB x TB tiles (TB = 16 for the matrix-core engine, 8 or
// 16 for the vector-ALU engine).  A tile that a wave is working on lives in
// registers, spread over the 64 lanes in the accumulator layout of the 16x16
// MFMA instructions, so a tile update can feed the matrix cores directly and
// the diagonal-tile solvers can work on the same registers.
//
// Accumulator layouts (measured on gfx950 with an in-bounds probe):
//   v_mfma_f64_16x16x4f64 : lane l holds rows (l>>4) + 4r, r = 0..3, column l&15
//   v_mfma_f32_16x16x4f32 / _16x16x16{f16,bf16}: rows 4(l>>4) + r, column l&15
// A operand (16 x K slice): lane l holds A[l&15][k-block(l>>4)];
// B operand (K x 16 slice): lane l holds B[k-block(l>>4)][l&15].
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "tla_internal.h"

namespace tla {

#define TLA_DI __device__ __forceinline__

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s4 __attribute__((ext_vector_type(4)));
typedef _Float16 h4 __attribute__((ext_vector_type(4)));

enum Engine { ENG_VALU = 0, ENG_MFMA = 1, ENG_MFMA_F16 = 2, ENG_MFMA_BF16 = 3 };

TLA_DI int lane_id() { return threadIdx.x & 63; }
TLA_DI int wave_id() { return threadIdx.x >> 6; }

// Orders LDS traffic between lanes of one wavefront: the LDS serves one
// wave's requests in issue order, so waiting for the outstanding ones and
// stopping the compiler from moving memory accesses across is enough.
TLA_DI void wave_fence() { asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory"); }

// --------------------------------------------------------------- views
// LDS-qualified element type: accesses through it compile to ds_read /
// ds_write rather than flat (generic) memory instructions.
template <class T>
using lds_t = __attribute__((address_space(3))) T;
template <class T>
TLA_DI lds_t<T>* to_lds(T* p) { return (lds_t<T>*)p; }
// global-memory-qualified element type (global_load / global_store)
template <class T>
using gbl_t = __attribute__((address_space(1))) T;
template <class T>
TLA_DI gbl_t<T>* to_gbl(T* p) { return (gbl_t<T>*)p; }
template <class T>
TLA_DI const gbl_t<T>* to_gbl(const T* p) { return (const gbl_t<T>*)p; }

// Strided matrix view: element (i, j) at p[i*rs + j*cs].  Column-major
// storage with leading dimension ld is (rs, cs) = (1, ld); t() transposes.
// LDS = true for matrices in LDS, false for global memory.
template <class T, bool LDS = true>
struct View {
  using P = std::conditional_t<LDS, lds_t<T>*, gbl_t<T>*>;
  P p;
  int rs, cs;
  TLA_DI T operator()(int i, int j) const { return p[i * rs + j * cs]; }
  TLA_DI auto& at(int i, int j) const { return p[i * rs + j * cs]; }
  TLA_DI void store(int i, int j, T v) const { p[i * rs + j * cs] = v; }
  TLA_DI View sub(int i0, int j0) const { return View{p + i0 * rs + j0 * cs, rs, cs}; }
  TLA_DI View t() const { return View{p, cs, rs}; }
  // Makes this wave's stores visible to its other lanes before they read:
  // the LDS serves a wave in order; global stores need to complete first.
  TLA_DI void fence() const {
    if constexpr (!LDS) __threadfence_block();
  }
};
template <class T>
TLA_DI View<T, true> colmajor(T* p, int ld) { return View<T, true>{to_lds(p), 1, ld}; }
template <class T>
TLA_DI View<T, false> gcolmajor(T* p, int ld) { return View<T, false>{to_gbl(p), 1, ld}; }
// column-major view in LDS or (XG) in global memory
template <bool XG, class T>
TLA_DI View<T, !XG> xcolmajor(T* p, int ld) {
  if constexpr (XG) return gcolmajor(p, ld);
  else return colmajor(p, ld);
}

// ----------------------------------------------------------- fragments
template <class T> struct Frag;
template <> struct Frag<double> {
  typedef d4 acc;
  static TLA_DI int row(int g, int r) { return g + 4 * r; }
  static TLA_DI acc mma(double a, double b, acc c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
};
template <> struct Frag<float> {
  typedef f4 acc;
  static TLA_DI int row(int g, int r) { return 4 * g + r; }
  static TLA_DI acc mma(float a, float b, acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
};

// A TB x TB tile in registers: EPL elements per lane.
//   TB = 16: lane l holds column l&15, rows Frag<T>::row(l>>4, r), r < 4
//   TB =  8: lane l holds column l&7,  row l>>3
template <class T, int TB>
struct Tile {
  static constexpr int EPL = TB * TB / 64;
  T v[EPL];
};

template <class T, int TB>
TLA_DI int trow(int lane, int r) {
  if constexpr (TB == 16) return Frag<T>::row(lane >> 4, r);
  else return lane >> 3;
}
template <int TB>
TLA_DI int tcol(int lane) { return lane & (TB - 1); }

template <class T, int TB, class V>
TLA_DI void tload(Tile<T, TB>& c, const V& M) {
  const int l = lane_id(), j = tcol<TB>(l);
#pragma unroll
  for (int r = 0; r < Tile<T, TB>::EPL; ++r) c.v[r] = M(trow<T, TB>(l, r), j);
}
template <class T, int TB, class V>
TLA_DI void tstore(const Tile<T, TB>& c, const V& M) {
  const int l = lane_id(), j = tcol<TB>(l);
#pragma unroll
  for (int r = 0; r < Tile<T, TB>::EPL; ++r) M.store(trow<T, TB>(l, r), j, c.v[r]);
  M.fence();
}
template <class T, int TB>
TLA_DI void tzero(Tile<T, TB>& c) {
#pragma unroll
  for (int r = 0; r < Tile<T, TB>::EPL; ++r) c.v[r] = T(0);
}

// ------------------------------------------------------ tile products
// c -= A * B for TB x TB operand views A, B (already offset to the tile).
template <class T, int TB, int ENG>
struct Gemm;

// Matrix cores in the working precision (f64 16x16x4 or f32 16x16x4).
// load() fetches one step's operand fragments, mma() consumes them.
template <class T>
struct Gemm<T, 16, ENG_MFMA> {
  struct F { T a[4], b[4]; };
  template <class VA, class VB>
  static TLA_DI void load(F& f, const VA& A, const VB& B) {
    const int l = lane_id(), i = l & 15, kq = l >> 4;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      f.a[kk] = -A(i, 4 * kk + kq);
      f.b[kk] = B(4 * kk + kq, i);
    }
  }
  static TLA_DI void mma(Tile<T, 16>& c, const F& f) {
    typename Frag<T>::acc acc = {c.v[0], c.v[1], c.v[2], c.v[3]};
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = Frag<T>::mma(f.a[kk], f.b[kk], acc);
    c.v[0] = acc[0]; c.v[1] = acc[1]; c.v[2] = acc[2]; c.v[3] = acc[3];
  }
  template <class VA, class VB>
  static TLA_DI void sub(Tile<T, 16>& c, const VA& A, const VB& B) {
    F f;
    load(f, A, B);
    mma(c, f);
  }
};

// Matrix cores in FP16 / BF16 with FP32 accumulation (FP32 working precision
// only): the operands are rounded to the 16-bit type, K = 16 in one step.
template <>
struct Gemm<float, 16, ENG_MFMA_F16> {
  struct F { h4 a, b; };
  template <class VA, class VB>
  static TLA_DI void load(F& f, const VA& A, const VB& B) {
    const int l = lane_id(), i = l & 15, kq = l >> 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      f.a[e] = (_Float16)(-A(i, 4 * kq + e));
      f.b[e] = (_Float16)(B(4 * kq + e, i));
    }
  }
  static TLA_DI void mma(Tile<float, 16>& c, const F& f) {
    f4 acc = {c.v[0], c.v[1], c.v[2], c.v[3]};
    acc = __builtin_amdgcn_mfma_f32_16x16x16f16(f.a, f.b, acc, 0, 0, 0);
    c.v[0] = acc[0]; c.v[1] = acc[1]; c.v[2] = acc[2]; c.v[3] = acc[3];
  }
  template <class VA, class VB>
  static TLA_DI void sub(Tile<float, 16>& c, const VA& A, const VB& B) {
    F f;
    load(f, A, B);
    mma(c, f);
  }
};
template <>
struct Gemm<float, 16, ENG_MFMA_BF16> {
  struct F { s4 a, b; };
  template <class VA, class VB>
  static TLA_DI void load(F& f, const VA& A, const VB& B) {
    const int l = lane_id(), i = l & 15, kq = l >> 4;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      f.a[e] = __builtin_bit_cast(short, (__bf16)(-A(i, 4 * kq + e)));
      f.b[e] = __builtin_bit_cast(short, (__bf16)(B(4 * kq + e, i)));
    }
  }
  static TLA_DI void mma(Tile<float, 16>& c, const F& f) {
    f4 acc = {c.v[0], c.v[1], c.v[2], c.v[3]};
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(f.a, f.b, acc, 0, 0, 0);
    c.v[0] = acc[0]; c.v[1] = acc[1]; c.v[2] = acc[2]; c.v[3] = acc[3];
  }
  template <class VA, class VB>
  static TLA_DI void sub(Tile<float, 16>& c, const VA& A, const VB& B) {
    F f;
    load(f, A, B);
    mma(c, f);
  }
};

// Vector ALU: each lane accumulates its own elements, k outermost.
template <class T, int TB>
struct Gemm<T, TB, ENG_VALU> {
  template <class VA, class VB>
  static TLA_DI void sub(Tile<T, TB>& c, const VA& A, const VB& B) {
    const int l = lane_id(), j = tcol<TB>(l);
#pragma unroll 4
    for (int k = 0; k < TB; ++k) {
      const T b = B(k, j);
#pragma unroll
      for (int r = 0; r < Tile<T, TB>::EPL; ++r) c.v[r] -= A(trow<T, TB>(l, r), k) * b;
    }
  }
};

// c -= sum_{K = k0}^{k1 - 1} fa(K) * fb(K), where fa / fb return the operand
// views of step K.  (Fetching step K + 1's fragments ahead of step K's
// products was measured slower: it raised register use and lowered the
// number of resident waves.)
template <class G, class Tl, class FA, class FB>
TLA_DI void gemm_sum(Tl& c, int k0, int k1, const FA& fa, const FB& fb) {
  for (int K = k0; K < k1; ++K) G::sub(c, fa(K), fb(K));
}

// ------------------------------------------------------ tile solvers
// All solvers run on one wavefront; `buf` is that wave's private LDS scratch
// of at least 3*TB elements.

// Triangular Sylvester on one tile:  Lt X + X Ut = c  (Lt lower, Ut upper,
// TB x TB views), overwriting c with X.  Element (i, j) is final once every
// (k, j), k < i and (i, k), k < j is; all elements on the anti-diagonal
// i + j = s are finalised together and then subtract their contribution
// from the elements below them in their column and right of them in their
// row.  Elements with i >= ni or j >= nj (padding) are forced to zero.
//
// The strictly triangular parts of Lt and Ut are first staged in the wave's
// scratch and the broadcast vectors are zeroed, so that the update of every
// step needs no test: a coefficient outside the strict triangle is zero, and
// a broadcast value not yet produced is zero.  One LDS fence per
// anti-diagonal: values finalised for step s + 1 are published at the end of
// step s, after this step's reads (the LDS serves a wave in order).
template <class T, int TB, class VL, class VU>
TLA_DI void tile_sylv(Tile<T, TB>& c, const VL& Lt, const VU& Ut, lds_t<T>* buf, int ni, int nj) {
  const int l = lane_id(), j = tcol<TB>(l);
  constexpr int E = Tile<T, TB>::EPL;
  constexpr int LD = TB + 1;
  lds_t<T>* colbuf = buf;              // colbuf[j] = element finalised in column j this step
  lds_t<T>* rowbuf = buf + TB;         // rowbuf[i] = element finalised in row i this step
  lds_t<T>* Ls = buf + 2 * TB;         // strictly lower part of Lt
  lds_t<T>* Us = Ls + TB * LD;         // strictly upper part of Ut
  T rinv[E];
  const T ujj = Ut(j, j);
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = trow<T, TB>(l, r);
    const T lv = Lt(i, j), uv = Ut(i, j);
    Ls[i + j * LD] = i > j ? lv : T(0);
    Us[i + j * LD] = i < j ? uv : T(0);
    rinv[r] = (i < ni && j < nj) ? T(1) / (Lt(i, i) + ujj) : T(0);
  }
  if (l < TB) {
    colbuf[l] = T(0);
    rowbuf[l] = T(0);
  }
  wave_fence();
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (trow<T, TB>(l, r) + j == 0) {
      const T x = c.v[r] * rinv[r];
      c.v[r] = x;
      colbuf[0] = x;
      rowbuf[0] = x;
    }
  }
#pragma unroll 1
  for (int s = 0; s < 2 * TB - 1; ++s) {
    int k = s - j;
    k = k < 0 ? 0 : (k > TB - 1 ? TB - 1 : k);
    T lv[E], uv[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = trow<T, TB>(l, r);
      int k2 = s - i;
      k2 = k2 < 0 ? 0 : (k2 > TB - 1 ? TB - 1 : k2);
      lv[r] = Ls[i + k * LD];
      uv[r] = Us[k2 + j * LD];
    }
    wave_fence();
    const T xc = colbuf[j];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const T xr = rowbuf[trow<T, TB>(l, r)];
      c.v[r] -= lv[r] * xc;
      c.v[r] -= xr * uv[r];
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = trow<T, TB>(l, r);
      if (i + j == s + 1) {
        const T x = c.v[r] * rinv[r];
        c.v[r] = x;
        colbuf[j] = x;
        rowbuf[i] = x;
      }
    }
  }
  wave_fence();
}

// Upper Cholesky of a diagonal tile held in c (only j >= i is used/valid):
// unblocked right-looking.  Pivots of rows >= nv are padding (value 1).
// The first failing pivot (<= 0 or NaN) is reported as base + k + 1 into
// *info if *info is still 0.  Row k of the partly updated tile is final
// after step k - 1; its owners publish it, and after one fence every lane
// forms the pivot and the scaled row entries it needs itself.
template <class T, int TB>
TLA_DI void tile_potf2(Tile<T, TB>& c, lds_t<T>* buf, int nv, int base, lds_t<int>* info) {
  const int l = lane_id(), j = tcol<TB>(l);
  constexpr int E = Tile<T, TB>::EPL;
  lds_t<T>* rowk = buf;   // rowk[j] = a_kj after the updates of steps < k
#pragma unroll
  for (int r = 0; r < E; ++r)
    if (trow<T, TB>(l, r) == 0) rowk[j] = c.v[r];
#pragma unroll 1
  for (int k = 0; k < TB; ++k) {
    wave_fence();
    const T p = rowk[k];
    const T d = sqrt(p);
    const T rd = T(1) / d;
    const T xj = rowk[j] * rd;
    if (l == 0 && !(p > T(0)) && k < nv && *info == 0) *info = base + k + 1;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = trow<T, TB>(l, r);
      if (i == k) c.v[r] = (j == k) ? d : (j > k ? xj : c.v[r]);
      else if (i > k && j >= i) c.v[r] -= (rowk[i] * rd) * xj;
    }
    // row k + 1 is now final: publish it (reads of rowk above came first)
#pragma unroll
    for (int r = 0; r < E; ++r)
      if (trow<T, TB>(l, r) == k + 1) rowk[j] = c.v[r];
  }
  wave_fence();
}

// Left solve with the transpose of an upper-triangular diagonal tile:
// c := Xd^{-T} c  (forward substitution down every column).  Row k of the
// solution is final after step k - 1 and is published then.
template <class T, int TB, class VX>
TLA_DI void tile_trsm_ut(Tile<T, TB>& c, const VX& Xd, lds_t<T>* buf) {
  const int l = lane_id(), j = tcol<TB>(l);
  constexpr int E = Tile<T, TB>::EPL;
  T xrow[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = trow<T, TB>(l, r);
    if (i == 0) {
      c.v[r] = c.v[r] / Xd(0, 0);
      buf[j] = c.v[r];
    }
  }
#pragma unroll 1
  for (int k = 0; k < TB - 1; ++k) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = trow<T, TB>(l, r);
      const T raw = Xd(k, i);
      xrow[r] = i > k ? raw : T(0);
    }
    const T dk1 = Xd(k + 1, k + 1);
    wave_fence();
    const T y = buf[j];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = trow<T, TB>(l, r);
      if (i > k) c.v[r] -= xrow[r] * y;
      if (i == k + 1) {
        c.v[r] = c.v[r] / dk1;
        buf[j] = c.v[r];
      }
    }
  }
  wave_fence();
}

// Right solve with an upper-triangular diagonal tile: c := c Xd^{-1}
// (substitution along every row, left to right); column k of the solution
// is published when it becomes final.
template <class T, int TB, class VX>
TLA_DI void tile_trsm_right_u(Tile<T, TB>& c, const VX& Xd, lds_t<T>* buf) {
  const int l = lane_id(), j = tcol<TB>(l);
  constexpr int E = Tile<T, TB>::EPL;
  if (j == 0) {
    const T d0 = Xd(0, 0);
#pragma unroll
    for (int r = 0; r < E; ++r) {
      c.v[r] = c.v[r] / d0;
      buf[trow<T, TB>(l, r)] = c.v[r];
    }
  }
#pragma unroll 1
  for (int k = 0; k < TB - 1; ++k) {
    const T uraw = Xd(k, j);
    const T u = j > k ? uraw : T(0);
    const T dk1 = Xd(k + 1, k + 1);
    wave_fence();
    T y[E];
#pragma unroll
    for (int r = 0; r < E; ++r) y[r] = buf[trow<T, TB>(l, r)];
    if (j > k) {
#pragma unroll
      for (int r = 0; r < E; ++r) c.v[r] -= y[r] * u;
    }
    if (j == k + 1) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        c.v[r] = c.v[r] / dk1;
        buf[trow<T, TB>(l, r)] = c.v[r];
      }
    }
  }
  wave_fence();
}

}  // namespace tla
