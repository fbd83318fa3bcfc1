// Mixed precision with a splitting iteration as the low-precision solve
// (triangular Sylvester and Lyapunov equations, n <= 64).
//
// The refinement is the classical one of the other mixed kernels: FP64
// residual R = C - L X - X U, backward error eta, low-precision correction
// D solving L D + D U = R, X += D in FP64 (Lyapunov: U = L^T).  What differs
// is the low-precision solve.  Split L = D_L + N_L and U = D_U + N_U into
// diagonal and strictly triangular parts; with d_ij = l_ii + u_jj the
// equation is d .* Y + N_L Y + Y N_U = F, and the sweep
//     Y <- (F - N_L Y - Y N_U) ./ d
// is a pair of matrix products per step.  N_L and N_U are nilpotent, so the
// error of sweep k vanishes on the anti-diagonals i + j < k and the sweep is
// exact after 2n - 1 steps in exact arithmetic; when the strict triangles are
// small against the diagonal sums it contracts by about
// ||N_L|| + ||N_U|| over min d_ij per step and reaches the low precision's
// accuracy in a handful of sweeps.  Every sweep is dense tile products on the
// matrix cores with no dependent chain of divisions, so the low-precision
// solve is bound by matrix-core throughput instead of the latency of the
// substitution chain; FP64 has no such shortcut on this chip (FP64 matrix
// cores run at the FP64 vector rate), which is what lets the mixed path
// gain.  Sweeps stop when the largest change falls below the product
// precision; an iteration that does not get there within the sweep limit
// simply yields a poor correction, which the refinement's stall test turns
// into the FP64 fallback (a second launch of the in-place FP64 kernel).
//
// Products: BF16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32 accumulate)
// with every FP32 operand split into a BF16 head and tail and three products
// (head x head + head x tail + tail x head), about 16 significant bits; or
// FP32 matrix cores (v_mfma_f32_16x16x4f32).  The residual runs on the FP64
// matrix cores.
//
// Layout: one wavefront per 16-wide tile column J of the instance (NT waves
// for n <= 16 NT); its tiles of the iterate Y, the right-hand side and the
// solution (an FP32 head Xh and tail Xl whose sum is exact in FP64) stay in
// registers in the accumulator layout (lane l holds rows 4(l>>4) + r of
// column l&15), with the column's -N_U fragments.  The -N_L fragments, the
// same for every column, are built once into LDS.  The product Y N_U needs
// rows of Y, which the accumulator layout holds as columns: every sweep
// writes Y into LDS row-major and the row fragments are read back from there
// (double buffered, one barrier per sweep).  The same buffers hold Xh and Xl
// for the residual.
#include <hip/hip_runtime.h>

#include <climits>
#include <cmath>

#include "tla_host.h"
#include "tla_kernels.hpp"
#include "tla_mixed.hpp"

namespace tla {
namespace {

typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

enum { JE_BF16X3 = 0, JE_F32 = 1 };

constexpr int kJacLd = 68;  // row stride (floats) of the row-major LDS copies: 16-byte aligned rows

template <int NT>
constexpr int jac_rows() { return NT * 16; }
template <int NT>
constexpr int jac_buf_floats() { return jac_rows<NT>() * kJacLd; }

// Row sigma(m) fed to the FP64 matrix cores as A row m, so that their
// accumulator layout (row g + 4r in lane g*16 + col, register r) comes out
// in the FP32 one (row 4g + r).
TLA_DI int sigma(int m) { return 4 * (m & 3) + (m >> 2); }

// Every element access below loads from a clamped, always valid address of
// the referenced part and masks the value by a multiplication, not a
// select: a loaded value that is only used under a condition gets a branch
// around its load, and each such load then waits for its data before the
// next one is issued.  (A non-finite referenced element makes a masked-out
// product NaN, but such an instance is flagged non-finite and solved again
// in FP64.)
template <bool SYM>
struct JacOps {
  const double* L;
  int ldl;
  const double* U;  // unused when SYM (U = L^T)
  int ldu;
  const double* C;
  int ldc;
  int n;
  // l_ij for the lower triangle (0 elsewhere and outside n x n)
  TLA_DI double l(int i, int j) const {
    const int ic = i < n ? i : n - 1, jc = j < n ? j : n - 1;
    const double v = to_gbl(L)[(ic > jc ? ic : jc) + (size_t)(ic < jc ? ic : jc) * ldl];
    return v * ((i < n && j < n && i >= j) ? 1.0 : 0.0);
  }
  // u_ij for the upper triangle
  TLA_DI double u(int i, int j) const {
    if constexpr (SYM) {
      return l(j, i);
    } else {
      const int ic = i < n ? i : n - 1, jc = j < n ? j : n - 1;
      const double v = to_gbl(U)[(ic < jc ? ic : jc) + (size_t)(ic > jc ? ic : jc) * ldu];
      return v * ((i < n && j < n && i <= j) ? 1.0 : 0.0);
    }
  }
  // right-hand side (Lyapunov: symmetric, read from its lower triangle)
  TLA_DI double c(int i, int j) const {
    int ic = i < n ? i : n - 1, jc = j < n ? j : n - 1;
    if (SYM && ic < jc) { const int t = ic; ic = jc; jc = t; }
    const double v = to_gbl(C)[ic + (size_t)jc * ldc];
    return v * ((i < n && j < n) ? 1.0 : 0.0);
  }
};

TLA_DI void split_bf16(float x, __bf16& h, __bf16& t) {
  h = (__bf16)x;
  t = (__bf16)(x - (float)h);
}

// Operand fragments of one K step of a tile product.  BF16X3: a pair of
// 16-wide K tiles (K0, K1) per instruction, element e of lane group g being
// k = K0*16 + 4g + e (e < 4) or K1*16 + 4g + e - 4 (e >= 4), so that the
// accumulator-layout registers of the tiles (K0, J), (K1, J) are directly the
// B operand.  F32: one K tile per four instructions, instruction kk taking
// k = K*16 + 4g + kk.
template <int JE>
struct JFrag;
template <>
struct JFrag<JE_BF16X3> {
  bf8 h, t;
};
template <>
struct JFrag<JE_F32> {
  float v[4];
};

TLA_DI JFrag<JE_BF16X3> frag_bf16(const float (&v)[8]) {
  JFrag<JE_BF16X3> f;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    __bf16 h, t;
    split_bf16(v[e], h, t);
    f.h[e] = h;
    f.t[e] = t;
  }
  return f;
}
// head x head, head x tail and tail x head into three accumulators (three
// independent chains for the matrix cores), summed by the caller
struct Acc3 { f4 hh, ht, th; };
TLA_DI void mma3(const JFrag<JE_BF16X3>& a, const JFrag<JE_BF16X3>& b, Acc3& acc) {
  acc.hh = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.h, acc.hh, 0, 0, 0);
  acc.ht = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.h, b.t, acc.ht, 0, 0, 0);
  acc.th = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.t, b.h, acc.th, 0, 0, 0);
}
TLA_DI f4 mma4(const JFrag<JE_F32>& a, const JFrag<JE_F32>& b, f4 acc) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a.v[kk], b.v[kk], acc, 0, 0, 0);
  return acc;
}

// Number of K steps of the products over K tiles 0..kmax: pairs for BF16X3,
// single tiles for F32.
template <int JE>
constexpr int ksteps(int kmax) { return JE == JE_BF16X3 ? kmax / 2 + 1 : kmax + 1; }
// Index of the first -N_L fragment of row tile I in LDS (rows 0..I-1 before it).
template <int JE>
constexpr int nl_base(int I) { return I == 0 ? 0 : nl_base<JE>(I - 1) + ksteps<JE>(I - 1); }
template <int JE>
constexpr int nl_count(int nt) { return nl_base<JE>(nt); }

typedef __bf16 bf4 __attribute__((ext_vector_type(4)));

// max that keeps a NaN from either side (fmaxf drops it), so that a
// non-finite iterate is seen by the convergence test
TLA_DI float nan_max(float a, float b) { return (a != a || b <= a) ? a : b; }

// nl_base for a run-time row tile (wave-uniform)
template <int JE>
TLA_DI int nl_base_rt(int I) { return JE == JE_BF16X3 ? (I / 2) * (I / 2 + 1) + (I & 1) * (I / 2 + 1) : I * (I + 1) / 2; }

TLA_DI int wave_min_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
  return v;
}

// Three sums over the workgroup (lane shares in, totals out on every thread).
template <int NW>
TLA_DI void block_sum3(double a, double b, double c, double* red, double& ta, double& tb, double& tc) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o);
    b += __shfl_xor(b, o);
    c += __shfl_xor(c, o);
  }
  if (lane_id() == 0) { red[3 * wave_id()] = a; red[3 * wave_id() + 1] = b; red[3 * wave_id() + 2] = c; }
  __syncthreads();
  ta = tb = tc = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) { ta += red[3 * w]; tb += red[3 * w + 1]; tc += red[3 * w + 2]; }
}

// Per-wave state: the wave's tile column J = wave index.
template <int NT, int JE>
struct JacState {
  static constexpr int NS = ksteps<JE>(NT - 1);  // K steps of a full row
  f4 y[NT];          // iterate (accumulator layout)
  bf4 yh[NT], yt[NT];  // its BF16 head and tail (BF16X3: the B operand halves)
  f4 fd[NT];         // right-hand side divided by d
  f4 rv[NT];         // 1 / d_ij, zero outside n x n so that padding stays zero
  f4 xh[NT];         // solution, FP32 head
  f4 xl[NT];         // solution, FP32 tail
  JFrag<JE> nu[NS];  // -N_U fragments (B operand) of the column, K step s
};

TLA_DI void split4(const f4& y, bf4& h, bf4& t) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    __bf16 a, b;
    split_bf16(y[e], a, b);
    h[e] = a;
    t[e] = b;
  }
}

// Row-major FP32 copy of the wave's column of an accumulator-layout matrix
// into LDS (row stride kJacLd).
template <int NT>
TLA_DI void put_rows(float* buf, const f4 (&m)[NT]) {
  const int l = lane_id(), g = l >> 4, c = l & 15, J = wave_id();
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) buf[(I * 16 + 4 * g + r) * kJacLd + J * 16 + c] = m[I][r];
}

// Four consecutive row elements from the FP32 copy: row i, columns k0..k0+3.
TLA_DI f4 get4(const float* buf, int i, int k0) {
  return *reinterpret_cast<const f4*>(buf + i * kJacLd + k0);
}

// BF16 row copies in fragment order: for row i, K pair p and lane group g,
// the 8 elements (tile 2p: columns 4g..4g+3, tile 2p+1: the same) are 16
// contiguous bytes, so the A fragment of Y(I, 2p..2p+1) is one read; the
// heads fill the first plane, the tails the second.
template <int NT>
constexpr int n_pairs() { return (NT + 1) / 2; }
template <int NT>
TLA_DI int frag_off(int i, int p, int g) { return ((i * n_pairs<NT>() + p) * 4 + g) * 16; }
template <int NT>
constexpr int plane_bytes() { return NT * 16 * n_pairs<NT>() * 64; }

// Writes tile (I, J = this wave) of the iterate into the BF16 row copies.
template <int NT>
TLA_DI void put_tile_bf16(unsigned char* buf, int I, const bf4& h, const bf4& t) {
  const int l = lane_id(), g = l >> 4, c = l & 15, J = wave_id();
  const int p = J >> 1, e = 4 * (J & 1) + (c & 3), gr = c >> 2;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int off = frag_off<NT>(I * 16 + 4 * g + r, p, gr) + 2 * e;
    *reinterpret_cast<__bf16*>(buf + off) = h[r];
    *reinterpret_cast<__bf16*>(buf + plane_bytes<NT>() + off) = t[r];
  }
}
template <int NT>
TLA_DI JFrag<JE_BF16X3> get_frag_bf16(const unsigned char* buf, int i, int p) {
  const int off = frag_off<NT>(i, p, lane_id() >> 4);
  JFrag<JE_BF16X3> f;
  f.h = *reinterpret_cast<const bf8*>(buf + off);
  f.t = *reinterpret_cast<const bf8*>(buf + plane_bytes<NT>() + off);
  return f;
}

// -N_L fragments in LDS: fragment f of lane l at nlf[f * 64 + l].
template <int JE>
TLA_DI JFrag<JE> get_nl(const JFrag<JE>* nlf, int f) { return nlf[f * 64 + lane_id()]; }

// One sweep Y <- Fd + (-N_L Y - Y N_U) ./ d over the wave's column.  The rows
// go from the first to the last and the column fragments Y(K, J), K < I, are
// already this sweep's (Gauss-Seidel along the column; the strictly lower
// part of the diagonal tile and the row fragments Y(I, K) of the other
// columns, read from `cur`, are the previous sweep's).  Each updated tile is
// written to `nxt` for the next sweep.  Accumulates this lane's largest
// change and largest new value (max-abs).
template <int NT, int JE>
TLA_DI void sweep(JacState<NT, JE>& s, const JFrag<JE>* nlf, const unsigned char* cur, unsigned char* nxt, int nt,
                  float& dmax, float& ymax) {
  constexpr int NS = JacState<NT, JE>::NS;
  const int l = lane_id(), g = l >> 4, c = l & 15, J = wave_id();
#pragma unroll
  for (int I = 0; I < NT; ++I) {
    if (I >= nt) continue;
    f4 acc = {0.f, 0.f, 0.f, 0.f};
    Acc3 a3 = {acc, acc, acc};
    // -N_L Y: K = 0..I
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      if (st >= ksteps<JE>(I)) continue;
      if constexpr (JE == JE_BF16X3) {
        const int K0 = 2 * st, K1 = K0 + 1 <= I ? K0 + 1 : K0;  // (A is zero in the second half then)
        JFrag<JE> b;
        b.h = __builtin_shufflevector(s.yh[K0], s.yh[K1], 0, 1, 2, 3, 4, 5, 6, 7);
        b.t = __builtin_shufflevector(s.yt[K0], s.yt[K1], 0, 1, 2, 3, 4, 5, 6, 7);
        mma3(get_nl<JE>(nlf, nl_base<JE>(I) + st), b, a3);
      } else {
        JFrag<JE> b;
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) b.v[kk] = s.y[st][kk];
        acc = mma4(get_nl<JE>(nlf, nl_base<JE>(I) + st), b, acc);
      }
    }
    // -Y N_U: K = 0..J, row fragments Y(I, K) from the previous sweep's copy
#pragma unroll
    for (int st = 0; st < NS; ++st) {
      if (st >= ksteps<JE>(J)) continue;
      if constexpr (JE == JE_BF16X3) {
        mma3(get_frag_bf16<NT>(cur, I * 16 + c, st), s.nu[st], a3);
      } else {
        JFrag<JE> a;
        const f4 a0 = get4(reinterpret_cast<const float*>(cur), I * 16 + c, st * 16 + 4 * g);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) a.v[kk] = a0[kk];
        acc = mma4(a, s.nu[st], acc);
      }
    }
    if constexpr (JE == JE_BF16X3) acc = a3.hh + (a3.ht + a3.th);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float yn = fmaf(acc[r], s.rv[I][r], s.fd[I][r]);
      dmax = nan_max(dmax, fabsf(yn - s.y[I][r]));
      ymax = nan_max(ymax, fabsf(yn));
      s.y[I][r] = yn;
    }
    if constexpr (JE == JE_BF16X3) {
      split4(s.y[I], s.yh[I], s.yt[I]);
      put_tile_bf16<NT>(nxt, I, s.yh[I], s.yt[I]);
    } else {
      float* nf = reinterpret_cast<float*>(nxt);
#pragma unroll
      for (int r = 0; r < 4; ++r) nf[(I * 16 + 4 * g + r) * kJacLd + J * 16 + c] = s.y[I][r];
    }
    compiler_fence();  // one row's fragments live at a time
  }
}

// Largest value over the wavefront (NaN if any lane holds one), on every
// lane: prefix maxima along each row of 16 lanes by DPP row shifts, then
// across rows by the row broadcasts, read from the last lane.
template <int CTRL, int ROW_MASK>
TLA_DI float dpp_max_step(float v) {
  const int o = __builtin_amdgcn_update_dpp(__builtin_bit_cast(int, v), __builtin_bit_cast(int, v), CTRL, ROW_MASK,
                                            0xf, false);
  return nan_max(v, __builtin_bit_cast(float, o));
}
TLA_DI float wave_max(float v) {
  v = dpp_max_step<0x111, 0xf>(v);  // row_shr:1
  v = dpp_max_step<0x112, 0xf>(v);  // row_shr:2
  v = dpp_max_step<0x114, 0xf>(v);  // row_shr:4
  v = dpp_max_step<0x118, 0xf>(v);  // row_shr:8
  v = dpp_max_step<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
  v = dpp_max_step<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), 63));
}

// Low-precision solve of d .* Y + N_L Y + Y N_U = F from Y = F ./ d
// (s.fd holds F ./ d).  buf0 / buf1: the two LDS row copies (double
// buffered); red: 2 * NT floats.  Returns false when the iterate is not
// finite.
template <int NT, int JE>
TLA_DI bool jacobi_solve(JacState<NT, JE>& s, const JFrag<JE>* nlf, float* buf0, float* buf1, float* red, int nt,
                         float tol, int max_sweeps, int& sweeps) {
  unsigned char* cur = reinterpret_cast<unsigned char*>(buf0);
  unsigned char* nxt = reinterpret_cast<unsigned char*>(buf1);
  if constexpr (JE == JE_BF16X3 && NT % 2 == 1) {
    // the second tile of the last pair does not exist: its half of every row
    // fragment must read as zero in both copies (the residual's FP32 rows
    // share the buffers)
    for (int e = threadIdx.x; e < 2 * jac_buf_floats<NT>(); e += blockDim.x) buf0[e] = 0.f;
    __syncthreads();
  }
#pragma unroll
  for (int I = 0; I < NT; ++I) {
    s.y[I] = s.fd[I];
    if constexpr (JE == JE_BF16X3) {
      split4(s.y[I], s.yh[I], s.yt[I]);
      put_tile_bf16<NT>(cur, I, s.yh[I], s.yt[I]);
    }
  }
  if constexpr (JE != JE_BF16X3) put_rows<NT>(reinterpret_cast<float*>(cur), s.y);
  __syncthreads();
  bool finite = true;
  for (int k = 0; k < max_sweeps; ++k) {
    float dmax = 0.f, ymax = 0.f;
    sweep(s, nlf, cur, nxt, nt, dmax, ymax);
    dmax = wave_max(dmax);
    ymax = wave_max(ymax);
    if (lane_id() == 0) { red[2 * wave_id()] = dmax; red[2 * wave_id() + 1] = ymax; }
    __syncthreads();
    float dm = 0.f, ym = 0.f;
#pragma unroll
    for (int w = 0; w < NT; ++w) { dm = nan_max(dm, red[2 * w]); ym = nan_max(ym, red[2 * w + 1]); }
    unsigned char* t = cur; cur = nxt; nxt = t;
    ++sweeps;
    if (!(dm == dm) || !(ym <= 3.0e38f)) { finite = false; break; }
    if (dm <= tol * ym) break;
    __syncthreads();  // every wave has read red before it is written again
  }
  return finite;
}

// The FP64 residual of the wave's column: R = C - L X - X U with X = Xh + Xl
// (row copies of Xh / Xl in buf0 / buf1).  The residual, rounded to FP32 and
// divided by d, becomes the next right-hand side (s.fd).  Accumulates this
// lane's shares of sum R^2 and sum X^2.
template <int NT, int JE, bool SYM>
TLA_DI void residual(JacState<NT, JE>& s, const JacOps<SYM>& op, const float* buf0, const float* buf1, int n,
                     int nt, double& sr, double& sx) {
  // The residual runs inside the refinement loop: an opaque zero in the
  // operand coordinates keeps the compiler from hoisting the 64-bit addresses
  // and bounds masks of every operand load out of that loop (they would all
  // stay live and spill).
  int z;
  asm volatile("v_mov_b32 %0, 0" : "=v"(z));
  const int l = lane_id(), g = (l >> 4) + z, c = l & 15, J = wave_id();
  const int rs = sigma(c);
#pragma unroll
  for (int I = 0; I < NT; ++I) {
    if (I >= nt) continue;
    // two independent accumulations (C - L X and - X U) for the matrix cores
    d4 acc, acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] = op.c(I * 16 + 4 * g + r, J * 16 + c);
    // - L X, K = 0..I (L rows permuted by sigma: the output lands in the FP32 layout)
#pragma unroll
    for (int K = 0; K < NT; ++K) {
      if (K > I) continue;
      double a[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) a[kk] = op.l(I * 16 + rs, K * 16 + 4 * g + kk);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double b = double(s.xh[K][kk]) + double(s.xl[K][kk]);
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(-a[kk], b, acc, 0, 0, 0);
      }
    }
    // - X U, K = 0..J (rows of X from the LDS copies)
#pragma unroll
    for (int K = 0; K < NT; ++K) {
      if (K > J) continue;
      double b[4];
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) b[kk] = op.u(K * 16 + 4 * g + kk, J * 16 + c);
      const f4 h = get4(buf0, I * 16 + rs, K * 16 + 4 * g), t = get4(buf1, I * 16 + rs, K * 16 + 4 * g);
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        const double a = -(double(h[kk]) + double(t[kk]));
        acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b[kk], acc2, 0, 0, 0);
      }
    }
    acc += acc2;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const double x = double(s.xh[I][r]) + double(s.xl[I][r]);
      sr += acc[r] * acc[r];
      sx += x * x;
      s.fd[I][r] = float(acc[r]) * s.rv[I][r];
    }
    // keeps the next tile's operand loads from being hoisted above this one's
    // products (they would all be live at once)
    compiler_fence();
  }
}

// Row copies of the solution into buf0 / buf1; for the Lyapunov equation it
// is first made exactly symmetric (every element above the diagonal takes its
// mirror below).
template <int NT, int JE, bool SYM>
TLA_DI void put_solution_rows(JacState<NT, JE>& s, float* buf0, float* buf1) {
  put_rows<NT>(buf0, s.xh);
  put_rows<NT>(buf1, s.xl);
  __syncthreads();
  if constexpr (SYM) {
    const int l = lane_id(), g = l >> 4, c = l & 15;
    const int j = wave_id() * 16 + c;
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * 16 + 4 * g + r;
        if (i < j) {
          s.xh[I][r] = buf0[j * kJacLd + i];
          s.xl[I][r] = buf1[j * kJacLd + i];
        }
      }
    __syncthreads();
    put_rows<NT>(buf0, s.xh);
    put_rows<NT>(buf1, s.xl);
    __syncthreads();
  }
}

// LDS of one instance: two row-major buffers, the -N_L fragments, reduction
// cells (2 NT floats, NT + 2 doubles) and the info cell.
template <int NT, int JE>
constexpr size_t jacobi_lds() {
  return 2 * (size_t)jac_buf_floats<NT>() * sizeof(float) + (size_t)nl_count<JE>(NT) * 64 * sizeof(JFrag<JE>) +
         2 * NT * sizeof(float) + 16 + (3 * NT + 2) * sizeof(double) + 16;
}

template <int NT, int JE, bool SYM>
TLA_DI void jacobi_mixed_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  constexpr int NS = JacState<NT, JE>::NS;
  int n;
  if (!validate(in, g.n_max, n)) return;
  const int nt = (n + 15) / 16;
  const int l = lane_id(), gq = l >> 4, c = l & 15, w = wave_id();
  float* buf0 = reinterpret_cast<float*>(smem);
  float* buf1 = buf0 + jac_buf_floats<NT>();
  JFrag<JE>* nlf = reinterpret_cast<JFrag<JE>*>(buf1 + jac_buf_floats<NT>());
  float* red = reinterpret_cast<float*>(nlf + nl_count<JE>(NT) * 64);
  double* dred = reinterpret_cast<double*>((reinterpret_cast<uintptr_t>(red + 2 * NT) + 15) & ~uintptr_t(15));
  int* s_info = reinterpret_cast<int*>(dred + 3 * NT + 2);

  const JacOps<SYM> op{in.a, in.lda, SYM ? nullptr : in.b, in.ldb, in.c, in.ldc, n};
  RefineState st{INFINITY, INFINITY, 0, 0};
  JacState<NT, JE> s;
  const int J = w, j = J * 16 + c;
  constexpr int EPF = JE == JE_BF16X3 ? 8 : 4;  // fragment elements per lane
  // Set-up.  Every global load comes first, so that all of them are in
  // flight together: the diagonals, the right-hand side of the wave's column,
  // the strict-triangle fragments (wave w builds the -N_L fragments of row
  // tile w and the -N_U fragments of its column).
  const double ujj = op.u(j, j), ljj = op.l(j, j);
  double lii[NT][4], cv[NT][4], nlx[NS][EPF], nux[NS][EPF];
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I * 16 + 4 * gq + r;
      lii[I][r] = op.l(i, i);
      cv[I][r] = op.c(i, j);
    }
  const int iw = w * 16 + c;  // row of the -N_L fragments this lane builds
#pragma unroll
  for (int stp = 0; stp < NS; ++stp)
#pragma unroll
    for (int e = 0; e < EPF; ++e) {
      // element e of K step stp: column k of -N_L (row iw) and row k of -N_U (column j)
      const int K = JE == JE_BF16X3 ? 2 * stp + (e >> 2) : stp;
      const int k = JE == JE_BF16X3 ? K * 16 + 4 * gq + (e & 3) : stp * 16 + 4 * gq + e;
      const double xl = op.l(iw, k), xu = op.u(k, j);
      nlx[stp][e] = xl * ((K <= w && k < iw) ? 1.0 : 0.0);
      nux[stp][e] = xu * ((K <= J && k < j) ? 1.0 : 0.0);
    }
  // 1 / d_ij, zero denominators (FP64: info; FP32: breakdown), right-hand
  // side over d, squared norms (strict triangles from the fragments, the
  // diagonals once per column)
  int best = INT_MAX;
  int zero32 = 0;
  double sc = 0.0, sl = (gq == 0 && j < n) ? ljj * ljj : 0.0, su = (gq == 0 && j < n) ? ujj * ujj : 0.0;
#pragma unroll
  for (int I = 0; I < NT; ++I)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = I * 16 + 4 * gq + r;
      const bool in_nn = i < n && j < n;
      const bool live = in_nn && (!SYM || i >= j);
      const double d = lii[I][r] + ujj;
      if (live && d == 0.0) best = min(best, 1 + i + j * n);
      if (live && float(lii[I][r]) + float(ujj) == 0.f) zero32 = 1;
      const double keep = in_nn ? 1.0 : 0.0;  // padding: d = 1, 1/d scaled to 0
      s.rv[I][r] = float(keep / (d * keep + (1.0 - keep)));
      s.fd[I][r] = float(cv[I][r]) * s.rv[I][r];
      s.xl[I][r] = 0.f;
      sc += cv[I][r] * cv[I][r];
    }
  JFrag<JE> fr;
#pragma unroll
  for (int stp = 0; stp < NS; ++stp) {
    float vl[EPF], vu[EPF];
#pragma unroll
    for (int e = 0; e < EPF; ++e) {
      sl += nlx[stp][e] * nlx[stp][e];
      su += nux[stp][e] * nux[stp][e];
      vl[e] = float(-nlx[stp][e]);
      vu[e] = float(-nux[stp][e]);
    }
    if constexpr (JE == JE_BF16X3) {
      fr = frag_bf16(vl);
      s.nu[stp] = frag_bf16(vu);
    } else {
#pragma unroll
      for (int e = 0; e < 4; ++e) { fr.v[e] = vl[e]; s.nu[stp].v[e] = vu[e]; }
    }
    if (stp < ksteps<JE>(w)) nlf[(nl_base_rt<JE>(w) + stp) * 64 + l] = fr;
  }
  if (threadIdx.x == 0) { *s_info = INT_MAX; red[0] = 0.f; }
  // zero row copies: pair halves beyond the last tile are never written
  for (int e = threadIdx.x; e < 2 * jac_buf_floats<NT>(); e += blockDim.x) buf0[e] = 0.f;
  __syncthreads();
  best = wave_min_int(best);
  zero32 = __any(zero32) ? 1 : 0;
  if (lane_id() == 0) {
    if (best != INT_MAX) atomicMin(s_info, best);
    if (zero32) atomicOr(reinterpret_cast<int*>(red), 1);
  }
  double nc, nl, nu;
  block_sum3<NT>(sc, sl, su, dred, nc, nl, nu);  // (its barrier also publishes the fragments, info and flags)
  nc = sqrt(nc);
  nl = sqrt(nl);
  nu = sqrt(nu);
  const int info0 = *s_info == INT_MAX ? 0 : *s_info;
  if (nc - nc != 0.0 || nl - nl != 0.0 || nu - nu != 0.0) st.flags |= TLA_STAT_NONFINITE;
  if (*reinterpret_cast<int*>(red) != 0) st.flags |= TLA_STAT_BREAKDOWN;
  __syncthreads();  // red is reused by the sweeps
  const float tol = JE == JE_BF16X3 ? 4.0e-6f : 2.5e-7f;
  const int max_sweeps = 2 * 16 * NT;
  int sweeps = 0;
  if (info0 == 0 && st.flags == 0) {
    if (!jacobi_solve(s, nlf, buf0, buf1, red, nt, tol, max_sweeps, sweeps)) st.flags |= TLA_STAT_BREAKDOWN;
    __syncthreads();
    if (st.flags == 0) {
#pragma unroll
      for (int I = 0; I < NT; ++I) s.xh[I] = s.y[I];
      for (;;) {
        put_solution_rows<NT, JE, SYM>(s, buf0, buf1);
        double sr = 0.0, sx = 0.0;
        residual(s, op, buf0, buf1, n, nt, sr, sx);
        const double nr = sqrt(block_sum<NT>(sr, dred));
        const double nx = sqrt(block_sum<NT>(sx, dred));
        const double eta = nr / ((nl + nu) * nx + nc);
        if (refine_decide(st, eta, g.tau, g.max_iter)) break;
        if (!jacobi_solve(s, nlf, buf0, buf1, red, nt, tol, max_sweeps, sweeps)) {
          st.flags |= TLA_STAT_BREAKDOWN;
          break;
        }
        __syncthreads();
        // X += D in FP64, kept as an FP32 head and tail
#pragma unroll
        for (int I = 0; I < NT; ++I)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double x = double(s.xh[I][r]) + double(s.xl[I][r]) + double(s.y[I][r]);
            const float h = float(x);
            s.xh[I][r] = h;
            s.xl[I][r] = float(x - double(h));
          }
        ++st.it;
      }
    }
  }
  // converged: the FP64 solution into the caller's matrix (the full matrix,
  // symmetric for the Lyapunov equation); otherwise C stays for the FP64 pass
  if (info0 == 0 && (st.flags & TLA_STAT_CONVERGED)) {
    gbl_t<double>* Cg = to_gbl(in.c);
#pragma unroll
    for (int I = 0; I < NT; ++I)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int i = I * 16 + 4 * gq + r;
        if (i < n && j < n) Cg[i + (size_t)j * in.ldc] = double(s.xh[I][r]) + double(s.xl[I][r]);
      }
  }
  if (threadIdx.x == 0) *in.info = info0;
  write_stat(in, st);
}

template <int NT, int JE, bool SYM>
__global__ __launch_bounds__(NT * 64) __attribute__((amdgpu_waves_per_eu(2))) void k_jacobi_mixed(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  jacobi_mixed_body<NT, JE, SYM>(g, fetch_uniform(g, blockIdx.x), smem);
}

template <int JE, bool SYM>
KFn pick(int nt, size_t* lds, int* waves) {
  if (nt <= 1) { *lds = jacobi_lds<1, JE>(); *waves = 1; return reinterpret_cast<KFn>(&k_jacobi_mixed<1, JE, SYM>); }
  if (nt <= 2) { *lds = jacobi_lds<2, JE>(); *waves = 2; return reinterpret_cast<KFn>(&k_jacobi_mixed<2, JE, SYM>); }
  if (nt <= 4) { *lds = jacobi_lds<4, JE>(); *waves = 4; return reinterpret_cast<KFn>(&k_jacobi_mixed<4, JE, SYM>); }
  return nullptr;
}

}  // namespace

// Kernel, LDS bytes and waves per instance of the splitting-iteration mixed
// solve for (op, prec, n_max); null when not built (FP64, FP16 products,
// Cholesky, or n_max above kJacobiMaxN).
KFn jacobi_kernel(int op, int prec, int n_max, size_t* lds, int* waves) {
  if (n_max > kJacobiMaxN || n_max < 0) return nullptr;
  const int nt = n_max < 1 ? 1 : (n_max + 15) / 16;
  if (prec == TLA_MIXED_BF16) {
    if (op == TLA_TRSYL) return pick<JE_BF16X3, false>(nt, lds, waves);
    if (op == TLA_TRLYAP) return pick<JE_BF16X3, true>(nt, lds, waves);
  } else if (prec == TLA_MIXED_F32) {
    if (op == TLA_TRSYL) return pick<JE_F32, false>(nt, lds, waves);
    if (op == TLA_TRLYAP) return pick<JE_F32, true>(nt, lds, waves);
  }
  return nullptr;
}

}  // namespace tla
