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
#ifndef __HIPCC_RTC__  // (the run-time compiler provides the HIP device API itself)
#include <hip/hip_runtime.h>
#endif
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
// Orders this thread's LDS accesses in the compiled code only.  Enough between
// a wave's LDS writes and its later reads of other lanes' values: the LDS
// serves one wave's accesses in the order they were issued.
TLA_DI void compiler_fence() { asm volatile("" ::: "memory"); }

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
  // symmetric matrices in a View are mirrored by the caller, not on store
  static constexpr bool mirrors() { return false; }
  // Makes this wave's stores visible to its other lanes before they read:
  // the LDS serves a wave in order; global stores need to complete first.
  TLA_DI void fence() const {
    if constexpr (!LDS) __threadfence_block();
  }
};
// True for views of matrices in LDS.
template <class V> struct InLds : std::false_type {};
template <class T> struct InLds<View<T, true>> : std::true_type {};

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

// Views of global memory that can tell whether a whole 16 x 16 block lies
// inside the matrix and its referenced part (interior16()) offer raw(i, j),
// an unmasked load; a product whose two operands are interior reads them that
// way, and only edge and diagonal blocks pay for the clamping and selects.
template <class V, class = void>
struct HasRaw : std::false_type {};
template <class V>
struct HasRaw<V, std::void_t<decltype(std::declval<const V&>().interior16())>> : std::true_type {};

// Matrix cores in the working precision (f64 16x16x4 or f32 16x16x4).
// load() fetches one step's operand fragments, mma() consumes them.
template <class T>
struct Gemm<T, 16, ENG_MFMA> {
  struct F { T a[4], b[4]; };
  template <class VA, class VB>
  static TLA_DI void load(F& f, const VA& A, const VB& B) {
    const int l = lane_id(), i = l & 15, kq = l >> 4;
    if constexpr (HasRaw<VA>::value && HasRaw<VB>::value) {
      if (A.interior16() && B.interior16()) {
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          f.a[kk] = -A.raw(i, 4 * kk + kq);
          f.b[kk] = B.raw(4 * kk + kq, i);
        }
        return;
      }
    }
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
// products was measured slower, also with operands read through the caches:
// it raised register use and lowered the number of resident waves.)
template <class G, class Tl, class FA, class FB>
TLA_DI void gemm_sum(Tl& c, int k0, int k1, const FA& fa, const FB& fb) {
  for (int K = k0; K < k1; ++K) G::sub(c, fa(K), fb(K));
}

// ------------------------------------------------------ tile solvers
// All solvers run on one wavefront; `buf` is that wave's private LDS scratch
// of wave_scratch(TB) elements.
//
// The 16 x 16 solvers first move the tile out of the matrix-core layout into
// one where every lane owns a small contiguous piece: a 2 x 2 block for the
// Sylvester tile, a strip of 4 consecutive elements of one column (or row) for
// the triangular solves and the Cholesky factorisation.  Most of the dependent
// chain then runs inside a lane's registers and the lanes exchange values once
// per block step (15 block anti-diagonals, or 4 strips) instead of once per
// element step (31 anti-diagonals, or 16 rows); the tile goes back to the
// matrix-core layout at the end.  The 8 x 8 tiles (one element per lane) use
// element-wise schedules.

// ---- Sylvester tile:  Lt X + X Ut = c  (Lt lower, Ut upper), c := X.
// Element (i, j) depends on the elements above it in its column and left of
// it in its row; everything with i >= ni or j >= nj is padding, forced to 0.

// Element schedule (any TB): the anti-diagonal i + j = s is finalised at step
// s - 1 and subtracts its contribution from the elements below it in its
// column and right of it in its row.  The strict triangles of Lt and Ut are
// staged in the scratch and the broadcast vectors start at zero, so the
// update of every step needs no test: a coefficient outside the strict
// triangle is zero and a value not yet produced is zero.  One LDS fence per
// step: values finalised for step s + 1 are published at the end of step s,
// after this step's reads (the LDS serves a wave in order).
template <class T, int TB, class VL, class VU>
TLA_DI void tile_sylv_elem(Tile<T, TB>& c, const VL& Lt, const VU& Ut, lds_t<T>* buf, int ni, int nj) {
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

// 2 x 2 block schedule (TB = 16): lane l owns block (I, J) = (l >> 3, l & 7),
// elements (2I + a, 2J + b).  Block (I, J) obeys
//   L_II X_IJ + X_IJ U_JJ = C_IJ - sum_{K<I} L_IK X_KJ - sum_{K<J} X_IK U_KJ,
// a 2 x 2 Sylvester system solved in registers once the block anti-diagonal
// I + J - 1 has been subtracted.  Step D subtracts the blocks of anti-diagonal
// D (published in cb / rb) and finalises anti-diagonal D + 1.  A lane reads
// a coefficient block and its broadcast partner only at the steps where their
// product is nonzero (a quarter of them on average); the LDS reads of the
// other lanes are masked off, which lowers the LDS traffic of a full compute
// unit.
template <int TB>
TLA_DI int blk2_index(int i, int j) {  // element (i, j) of a tile stored as 2 x 2 blocks
  return 4 * ((TB / 2) * (i >> 1) + (j >> 1)) + 2 * (i & 1) + (j & 1);
}

// Coefficients one lane needs for the 2 x 2 block schedule: its block of Lt
// and of Ut and the diagonal blocks of its row and column.  Fetched apart from
// the solve so that callers can issue these loads before the tile's updates.
template <class T>
struct Blk2Coef {
  T lv[4], uv[4];
  T l00, l10, l11, u00, u01, u11;
};

template <class T, class VL, class VU>
TLA_DI Blk2Coef<T> blk2_fetch(const VL& Lt, const VU& Ut) {
  const int l = lane_id(), i0 = 2 * (l >> 3), j0 = 2 * (l & 7);
  Blk2Coef<T> k;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      k.lv[2 * a + b] = Lt(i0 + a, j0 + b);
      k.uv[2 * a + b] = Ut(i0 + a, j0 + b);
    }
  k.l00 = Lt(i0, i0);
  k.l10 = Lt(i0 + 1, i0);
  k.l11 = Lt(i0 + 1, i0 + 1);
  k.u00 = Ut(j0, j0);
  k.u01 = Ut(j0, j0 + 1);
  k.u11 = Ut(j0 + 1, j0 + 1);
  return k;
}

template <class T>
TLA_DI void tile_sylv_blk2(Tile<T, 16>& c, const Blk2Coef<T>& k, lds_t<T>* buf, int ni, int nj) {
  const int l = lane_id(), I = l >> 3, J = l & 7;
  lds_t<T>* Lb = buf;        // block (I, K) at 4 (8 I + K): Lt's block if K < I, else 0
  lds_t<T>* Ub = buf + 256;  // block (K, J) at 4 (8 K + J): Ut's block if K < J, else 0
  lds_t<T>* cb = buf + 512;  // cb[J]: block of column J finalised at the last step
  lds_t<T>* rb = buf + 544;  // rb[I]: block of row I finalised at the last step
  {
    const int lj = tcol<16>(l);
#pragma unroll
    for (int r = 0; r < 4; ++r) Lb[blk2_index<16>(trow<T, 16>(l, r), lj)] = c.v[r];
  }
  wave_fence();
  T x[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) x[e] = Lb[4 * l + e];
  // the reads above are served before these writes (same wave, LDS in order)
  const int i0 = 2 * I, j0 = 2 * J;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    Lb[4 * l + e] = J < I ? k.lv[e] : T(0);
    Ub[4 * l + e] = I < J ? k.uv[e] : T(0);
  }
  const T l00 = k.l00, l10 = k.l10, l11 = k.l11, u00 = k.u00, u01 = k.u01, u11 = k.u11;
  const bool r0 = i0 < ni, r1 = i0 + 1 < ni, c0 = j0 < nj, c1 = j0 + 1 < nj;
  const T q00 = (r0 && c0) ? T(1) / (l00 + u00) : T(0);
  const T q01 = (r0 && c1) ? T(1) / (l00 + u11) : T(0);
  const T q10 = (r1 && c0) ? T(1) / (l11 + u00) : T(0);
  const T q11 = (r1 && c1) ? T(1) / (l11 + u11) : T(0);
  // the 2 x 2 system by elements: (0,0), then (0,1) and (1,0), then (1,1)
  auto finalise = [&]() {
    const T y00 = x[0] * q00;
    const T y01 = (x[1] - y00 * u01) * q01;
    const T y10 = (x[2] - l10 * y00) * q10;
    const T y11 = (x[3] - l10 * y01 - y10 * u01) * q11;
    x[0] = y00; x[1] = y01; x[2] = y10; x[3] = y11;
  };
  wave_fence();
  if (l == 0) {
    finalise();
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      cb[e] = x[e];
      rb[e] = x[e];
    }
  }
#pragma unroll 1
  for (int D = 0; D < 14; ++D) {
    // a lane reads a block pair only when its product is nonzero: L_IK with
    // K = D - J < I (X_KJ finalised at the last step), U_K'J with K' = D - I < J
    const int K = D - J, K2 = D - I;
    T lk[4] = {T(0), T(0), T(0), T(0)}, uk[4] = {T(0), T(0), T(0), T(0)};
    T xc[4] = {T(0), T(0), T(0), T(0)}, xr[4] = {T(0), T(0), T(0), T(0)};
    compiler_fence();
    if (K >= 0 && K < I) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        lk[e] = Lb[4 * (8 * I + K) + e];
        xc[e] = cb[4 * J + e];
      }
    }
    if (K2 >= 0 && K2 < J) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        uk[e] = Ub[4 * (8 * K2 + J) + e];
        xr[e] = rb[4 * I + e];
      }
    }
    // c -= L_IK X_KJ + X_IK' U_K'J on row-major 2 x 2 blocks
    x[0] -= lk[0] * xc[0] + lk[1] * xc[2] + xr[0] * uk[0] + xr[1] * uk[2];
    x[1] -= lk[0] * xc[1] + lk[1] * xc[3] + xr[0] * uk[1] + xr[1] * uk[3];
    x[2] -= lk[2] * xc[0] + lk[3] * xc[2] + xr[2] * uk[0] + xr[3] * uk[2];
    x[3] -= lk[2] * xc[1] + lk[3] * xc[3] + xr[2] * uk[1] + xr[3] * uk[3];
    compiler_fence();
    if (I + J == D + 1) {
      finalise();
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        cb[4 * J + e] = x[e];
        rb[4 * I + e] = x[e];
      }
    }
  }
  wave_fence();
  // back to the matrix-core layout (the loop's reads of Lb were served first)
#pragma unroll
  for (int e = 0; e < 4; ++e) Lb[4 * l + e] = x[e];
  wave_fence();
  {
    const int lj = tcol<16>(l);
#pragma unroll
    for (int r = 0; r < 4; ++r) c.v[r] = Lb[blk2_index<16>(trow<T, 16>(l, r), lj)];
  }
  wave_fence();
}

// Two-phase interface: sylv_fetch issues the coefficient loads of a diagonal
// tile pair, sylv_solve solves the tile with them.
template <class VL, class VU>
struct ViewPair {
  VL L;
  VU U;
};

// Coefficient tiles outside LDS are fetched as two whole tiles (their loads
// read along columns) instead of the 14 gathered elements per lane of the 2 x 2
// block schedule, and staged through the wave's scratch when the solve starts.
template <class T>
struct Blk2Tiles {
  Tile<T, 16> L, U;
};

template <class T>
TLA_DI Blk2Coef<T> blk2_from_tiles(const Blk2Tiles<T>& t, lds_t<T>* buf) {
  constexpr int LD = 17;
  lds_t<T>* Ls = buf;
  lds_t<T>* Us = buf + 16 * LD;
  const int l = lane_id(), j = tcol<16>(l);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    Ls[trow<T, 16>(l, r) + j * LD] = t.L.v[r];
    Us[trow<T, 16>(l, r) + j * LD] = t.U.v[r];
  }
  compiler_fence();
  const Blk2Coef<T> k = blk2_fetch<T>(View<T, true>{Ls, 1, LD}, View<T, true>{Us, 1, LD});
  compiler_fence();  // served before the solver's first writes to the scratch
  return k;
}

template <class T, int TB, class VL, class VU>
TLA_DI auto sylv_fetch(const VL& Lt, const VU& Ut) {
  if constexpr (TB == 16 && InLds<VL>::value && InLds<VU>::value) {
    return blk2_fetch<T>(Lt, Ut);
  } else if constexpr (TB == 16) {
    Blk2Tiles<T> t;
    tload(t.L, Lt);
    tload(t.U, Ut);
    return t;
  } else {
    return ViewPair<VL, VU>{Lt, Ut};
  }
}

template <class T, int TB, class K>
TLA_DI void sylv_solve(Tile<T, TB>& c, const K& k, lds_t<T>* buf, int ni, int nj) {
  if constexpr (TB == 16 && std::is_same_v<K, Blk2Tiles<T>>) tile_sylv_blk2<T>(c, blk2_from_tiles<T>(k, buf), buf, ni, nj);
  else if constexpr (TB == 16) tile_sylv_blk2<T>(c, k, buf, ni, nj);
  else tile_sylv_elem<T, TB>(c, k.L, k.U, buf, ni, nj);
}

template <class T, int TB, class VL, class VU>
TLA_DI void tile_sylv(Tile<T, TB>& c, const VL& Lt, const VU& Ut, lds_t<T>* buf, int ni, int nj) {
  sylv_solve<T, TB>(c, sylv_fetch<T, TB>(Lt, Ut), buf, ni, nj);
}

// Square root of a pivot and its reciprocal for the Cholesky tiles, without
// the long dependent chains of a correctly rounded square root followed by a
// division: the hardware reciprocal square root estimate is refined by
// Newton-Raphson steps y <- y + y (1 - p y^2) / 2, the root s = p y is
// corrected once with its exact residual p - s^2 (fused multiply-add;
// Markstein's final step), and the reciprocal by one Newton step from y.
// Exact square roots (perfect squares) come out exact.
TLA_DI void pivot_root(double p, double& s, double& r) {
  double y = __builtin_amdgcn_rsq(p);
#pragma unroll
  for (int it = 0; it < 2; ++it) y = __builtin_fma(0.5 * y, __builtin_fma(-p * y, y, 1.0), y);
  s = p * y;
  s = __builtin_fma(__builtin_fma(-s, s, p), 0.5 * y, s);
  r = __builtin_fma(y, __builtin_fma(-s, y, 1.0), y);
}
TLA_DI void pivot_root(float p, float& s, float& r) {
  float y = __builtin_amdgcn_rsqf(p);
  y = __builtin_fmaf(0.5f * y, __builtin_fmaf(-p * y, y, 1.0f), y);
  s = p * y;
  s = __builtin_fmaf(__builtin_fmaf(-s, s, p), 0.5f * y, s);
  r = __builtin_fmaf(y, __builtin_fmaf(-s, y, 1.0f), y);
}

// ---- Upper Cholesky of a diagonal tile held in c (only j >= i is used and
// written; the strict lower part is left as it is).  Pivots of rows >= nv are
// padding (value 1).  The first failing pivot (<= 0 or NaN) is reported as
// base + k + 1 into *info if *info is still 0.  The diagonal is the square
// root of the pivot and a row is scaled by the reciprocal of its diagonal, as
// in the element recurrence (both from pivot_root).

// Element schedule, right-looking: row k of the partly updated tile is final
// after step k - 1; its owners publish it, and after one fence every lane
// reads the pivot and the row entries it needs (all reads of a step are
// issued together) and forms the step's values itself.
template <class T, int TB>
TLA_DI void tile_potf2_elem(Tile<T, TB>& c, lds_t<T>* buf, int nv, int base, lds_t<int>* info) {
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
    const T rj = rowk[j];
    T ri[E];
#pragma unroll
    for (int r = 0; r < E; ++r) ri[r] = rowk[trow<T, TB>(l, r)];
    const int inf0 = *info;
    T d, rd;
    pivot_root(p, d, rd);
    const T xj = rj * rd;
    if (l == 0 && !(p > T(0)) && k < nv && inf0 == 0) *info = base + k + 1;
    T pub = T(0);
    bool has = false;
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = trow<T, TB>(l, r);
      const T upd = c.v[r] - (ri[r] * rd) * xj;
      const T rowv = (j == k) ? d : (j > k ? xj : c.v[r]);
      c.v[r] = (i == k) ? rowv : ((i > k && j >= i) ? upd : c.v[r]);
      pub = (i == k + 1) ? c.v[r] : pub;
      has = has || i == k + 1;
    }
    // row k + 1 is now final: publish it (this step's reads were issued first)
    if (has) rowk[j] = pub;
  }
  wave_fence();
}

// 4-row strip schedule (TB = 16): lane (g, j) = (l >> 4, l & 15) holds rows
// 4g..4g+3 of column j.  Block step G: strip G has been updated by all
// earlier strips and is published; every lane reads the 4 x 4 diagonal block
// and factors it itself, solves its own column segment X_G,j = X_GG^{-T} A_G,j
// and, below strip G, the segments of the columns that match its rows, then
// subtracts X_G,i^T X_G,j from its strip.  Strip G + 1 publishes for the next
// step.
template <class T>
TLA_DI void tile_potf2_strip(Tile<T, 16>& c, lds_t<T>* buf, int nv, int base, lds_t<int>* info) {
  const int l = lane_id(), j = l & 15, g = l >> 4;
  constexpr int LD = 17;
  lds_t<T>* S = buf;  // the tile, column-major, leading dimension 17
#pragma unroll
  for (int r = 0; r < 4; ++r) S[trow<T, 16>(l, r) + j * LD] = c.v[r];
  compiler_fence();
  T a[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) a[e] = S[4 * g + e + j * LD];
  int bad = 0;
#pragma unroll 1
  for (int G = 0; G < 4; ++G) {
    const int o = 4 * G;
    T d[4][4], w[4], v[4][4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
#pragma unroll
      for (int q = p; q < 4; ++q) d[p][q] = S[o + p + (o + q) * LD];
      w[p] = S[o + p + j * LD];
    }
#pragma unroll
    for (int e = 0; e < 4; ++e)
#pragma unroll
      for (int p = 0; p < 4; ++p) v[e][p] = S[o + p + (4 * g + e) * LD];
    // X_GG: upper Cholesky of the diagonal block, rr[p] = 1 / x_pp
    T x[4][4], rr[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      T piv = d[p][p];
#pragma unroll
      for (int k = 0; k < p; ++k) piv -= x[k][p] * x[k][p];
      if (!(piv > T(0)) && o + p < nv && bad == 0) bad = base + o + p + 1;
      pivot_root(piv, x[p][p], rr[p]);
#pragma unroll
      for (int q = p + 1; q < 4; ++q) {
        T s = d[p][q];
#pragma unroll
        for (int k = 0; k < p; ++k) s -= x[k][p] * x[k][q];
        x[p][q] = s * rr[p];
      }
    }
    // own column segment y = X_GG^{-T} A_G,j
    T y[4];
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      T s = w[p];
#pragma unroll
      for (int k = 0; k < p; ++k) s -= x[k][p] * y[k];
      y[p] = s * rr[p];
    }
    if (g == G) {
#pragma unroll
      for (int e = 0; e < 4; ++e) a[e] = (o + e < j) ? y[e] : (o + e == j ? x[e][e] : a[e]);
    } else if (g > G) {
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        T z[4];
#pragma unroll
        for (int p = 0; p < 4; ++p) {
          T s = v[e][p];
#pragma unroll
          for (int k = 0; k < p; ++k) s -= x[k][p] * z[k];
          z[p] = s * rr[p];
        }
        T u = a[e];
#pragma unroll
        for (int p = 0; p < 4; ++p) u -= z[p] * y[p];
        a[e] = (4 * g + e <= j) ? u : a[e];
      }
    }
    if (g == G + 1) {
#pragma unroll
      for (int e = 0; e < 4; ++e) S[4 * g + e + j * LD] = a[e];
    }
    compiler_fence();
  }
  if (l == 0 && bad != 0 && *info == 0) *info = bad;
#pragma unroll
  for (int e = 0; e < 4; ++e) S[4 * g + e + j * LD] = a[e];
  compiler_fence();
#pragma unroll
  for (int r = 0; r < 4; ++r) c.v[r] = S[trow<T, 16>(l, r) + j * LD];
  compiler_fence();
}

template <class T, int TB>
TLA_DI void tile_potf2(Tile<T, TB>& c, lds_t<T>* buf, int nv, int base, lds_t<int>* info) {
  if constexpr (TB == 16) tile_potf2_strip<T>(c, buf, nv, base, info);
  else tile_potf2_elem<T, TB>(c, buf, nv, base, info);
}

// ---- Triangular solves with an upper-triangular diagonal tile Xd:
//   tile_trsm_ut:      c := Xd^{-T} c  (forward substitution down every column)
//   tile_trsm_right_u: c := c Xd^{-1}  (substitution along every row)
// Both solve Xd^T y = v for 16 independent vectors v (the columns, or the
// rows, of c).

// Element schedules (any TB): element k of every vector is final after step
// k - 1 and is published then.
template <class T, int TB, class VX>
TLA_DI void tile_trsm_ut_elem(Tile<T, TB>& c, const VX& Xd, lds_t<T>* buf) {
  const int l = lane_id(), j = tcol<TB>(l);
  constexpr int E = Tile<T, TB>::EPL;
  T xrow[E], rinv[E];
#pragma unroll
  for (int r = 0; r < E; ++r) {
    const int i = trow<T, TB>(l, r);
    rinv[r] = T(1) / Xd(i, i);
  }
#pragma unroll
  for (int r = 0; r < E; ++r) {
    if (trow<T, TB>(l, r) == 0) {
      c.v[r] = c.v[r] * rinv[r];
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
    wave_fence();
    const T y = buf[j];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const int i = trow<T, TB>(l, r);
      c.v[r] -= xrow[r] * y;
      if (i == k + 1) {
        c.v[r] = c.v[r] * rinv[r];
        buf[j] = c.v[r];
      }
    }
  }
  wave_fence();
}

template <class T, int TB, class VX>
TLA_DI void tile_trsm_right_u_elem(Tile<T, TB>& c, const VX& Xd, lds_t<T>* buf) {
  const int l = lane_id(), j = tcol<TB>(l);
  constexpr int E = Tile<T, TB>::EPL;
  const T rj = T(1) / Xd(j, j);
  if (j == 0) {
#pragma unroll
    for (int r = 0; r < E; ++r) {
      c.v[r] = c.v[r] * rj;
      buf[trow<T, TB>(l, r)] = c.v[r];
    }
  }
#pragma unroll 1
  for (int k = 0; k < TB - 1; ++k) {
    const T uraw = Xd(k, j);
    const T u = j > k ? uraw : T(0);
    wave_fence();
    T y[E];
#pragma unroll
    for (int r = 0; r < E; ++r) y[r] = buf[trow<T, TB>(l, r)];
#pragma unroll
    for (int r = 0; r < E; ++r) c.v[r] -= y[r] * u;
    if (j == k + 1) {
#pragma unroll
      for (int r = 0; r < E; ++r) {
        c.v[r] = c.v[r] * rj;
        buf[trow<T, TB>(l, r)] = c.v[r];
      }
    }
  }
  wave_fence();
}

// Strip schedule (TB = 16): lane (g, v) = (l >> 4, l & 15) holds elements
// 4g..4g+3 of vector v.  Block step G: strip G finishes with a 4 x 4 forward
// substitution in registers and publishes; the strips below subtract
// Xd^T(strip g, strip G) times it.  RIGHT selects rows of c as the vectors.
// A coefficient tile outside LDS is first copied into the wave's scratch
// (after the work tile) by one tile load whose element loads overlap; the
// strips then read it from there instead of waiting on memory at each step.
template <class T, class VX>
TLA_DI View<T, true> stage_coef_tile(const VX& Xd, lds_t<T>* buf) {
  constexpr int LD = 17;
  lds_t<T>* Xs = buf + 16 * LD;
  Tile<T, 16> xt;
  tload(xt, Xd);
  const int l = lane_id();
#pragma unroll
  for (int r = 0; r < 4; ++r) Xs[trow<T, 16>(l, r) + tcol<16>(l) * LD] = xt.v[r];
  compiler_fence();
  return View<T, true>{Xs, 1, LD};
}

template <class T, bool RIGHT, class VX>
TLA_DI void tile_trsv_strips(Tile<T, 16>& c, const VX& Xd, lds_t<T>* buf) {
  if constexpr (!InLds<VX>::value) {
    tile_trsv_strips<T, RIGHT>(c, stage_coef_tile<T>(Xd, buf), buf);
    return;
  }
  const int l = lane_id(), jc = tcol<16>(l), g = l >> 4, v = l & 15;
  constexpr int LD = 17;
  constexpr int rs = RIGHT ? LD : 1, cs = RIGHT ? 1 : LD;  // element e of vector v at e*rs + v*cs
  lds_t<T>* S = buf;
#pragma unroll
  for (int r = 0; r < 4; ++r) S[trow<T, 16>(l, r) + jc * LD] = c.v[r];
  T dg[4][4], rin[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = 0; b < a; ++b) dg[a][b] = Xd(4 * g + b, 4 * g + a);
    rin[a] = T(1) / Xd(4 * g + a, 4 * g + a);
  }
  compiler_fence();
  T y[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) y[a] = S[(4 * g + a) * rs + v * cs];
#pragma unroll
  for (int G = 0; G < 4; ++G) {
    if (g == G) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        T acc = y[a];
#pragma unroll
        for (int b = 0; b < a; ++b) acc -= dg[a][b] * y[b];
        y[a] = acc * rin[a];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) S[(4 * G + a) * rs + v * cs] = y[a];
    }
    if (G == 3) break;
    // Xd^T(4g + a, 4G + b) = Xd(4G + b, 4g + a), used by the strips g > G
    T cf[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) cf[a][b] = Xd(4 * G + b, 4 * g + a);
    compiler_fence();
    T z[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) z[b] = S[(4 * G + b) * rs + v * cs];
    if (g > G) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) y[a] -= cf[a][b] * z[b];
    }
  }
  compiler_fence();
#pragma unroll
  for (int r = 0; r < 4; ++r) c.v[r] = S[trow<T, 16>(l, r) + jc * LD];
  compiler_fence();
}

// Left solve with an upper-triangular diagonal tile: c := Xd^{-1} c (back
// substitution up every column), 16 x 16 tiles, strip schedule: lane (g, v)
// holds rows 4g..4g+3 of column v; strips are finished from the last one up,
// each with a 4 x 4 back substitution in registers, and the strips above
// subtract Xd(strip g, strip G) times the finished strip.
template <class T, class VX>
TLA_DI void tile_trsm_u(Tile<T, 16>& c, const VX& Xd, lds_t<T>* buf) {
  if constexpr (!InLds<VX>::value) {
    tile_trsm_u<T>(c, stage_coef_tile<T>(Xd, buf), buf);
    return;
  }
  const int l = lane_id(), jc = tcol<16>(l), g = l >> 4, v = l & 15;
  constexpr int LD = 17;
  lds_t<T>* S = buf;
#pragma unroll
  for (int r = 0; r < 4; ++r) S[trow<T, 16>(l, r) + jc * LD] = c.v[r];
  T dg[4][4], rin[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
#pragma unroll
    for (int b = a + 1; b < 4; ++b) dg[a][b] = Xd(4 * g + a, 4 * g + b);
    rin[a] = T(1) / Xd(4 * g + a, 4 * g + a);
  }
  compiler_fence();
  T y[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) y[a] = S[4 * g + a + v * LD];
#pragma unroll
  for (int G = 3; G >= 0; --G) {
    if (g == G) {
#pragma unroll
      for (int a = 3; a >= 0; --a) {
        T acc = y[a];
#pragma unroll
        for (int b = a + 1; b < 4; ++b) acc -= dg[a][b] * y[b];
        y[a] = acc * rin[a];
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) S[4 * G + a + v * LD] = y[a];
    }
    if (G == 0) break;
    // Xd(4g + a, 4G + b), used by the strips g < G
    T cf[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) cf[a][b] = Xd(4 * g + a, 4 * G + b);
    compiler_fence();
    T z[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) z[b] = S[4 * G + b + v * LD];
    if (g < G) {
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) y[a] -= cf[a][b] * z[b];
    }
  }
  compiler_fence();
#pragma unroll
  for (int r = 0; r < 4; ++r) c.v[r] = S[trow<T, 16>(l, r) + jc * LD];
  compiler_fence();
}

template <class T, int TB, class VX>
TLA_DI void tile_trsm_ut(Tile<T, TB>& c, const VX& Xd, lds_t<T>* buf) {
  if constexpr (TB == 16) tile_trsv_strips<T, false>(c, Xd, buf);
  else tile_trsm_ut_elem<T, TB>(c, Xd, buf);
}

template <class T, int TB, class VX>
TLA_DI void tile_trsm_right_u(Tile<T, TB>& c, const VX& Xd, lds_t<T>* buf) {
  if constexpr (TB == 16) tile_trsv_strips<T, true>(c, Xd, buf);
  else tile_trsm_right_u_elem<T, TB>(c, Xd, buf);
}

}  // namespace tla
