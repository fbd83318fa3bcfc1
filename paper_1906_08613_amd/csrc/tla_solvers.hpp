// Blocked algorithm variants for the three operations of the paper (Fig. 2):
// upper Cholesky X^T X = A, triangular Sylvester L X + X U = C and triangular
// Lyapunov L X + X L^T = S.
//
// The paper synthesises, for each operation, a family of loop-based blocked
// algorithms that are mathematically equivalent but differ in performance,
// and picks among them by autotuning (Generator structure paragraph; four
// variants for the Sylvester equation in the results paragraph).  The
// variants below are the partitioned-matrix-expression algorithms of the
// three operations, expressed over TB x TB tiles and scheduled on the NW
// wavefronts of one workgroup: tiles that do not depend on each other are
// handed to different waves between workgroup barriers.
//
// All routines work in place on a work matrix W in LDS (column-major, padded
// to nt*TB rows and columns with the padding already initialised) and read
// the triangular coefficients through views that return zero outside n.
#pragma once
#include "tla_tiles.hpp"

namespace tla {

// Per-workgroup context handed to the drivers.
template <class T>
struct Ctx {
  int n;              // order of this instance
  int nt;             // number of tiles per dimension, ceil(n / TB)
  lds_t<T>* wbuf;     // per-wave LDS scratch (this wave's slice)
  lds_t<int>* info;   // LDS cell for the instance's info (first failure wins)
};

// ======================================================= Cholesky X^T X = A
// Variants (upper factor, A_TL / A_TR / A_BR partition):
//   CHOL_RL  right-looking: factor A11, solve the row panel A12 := X11^{-T} A12,
//            update the trailing matrix A22 -= A12^T A12.
//   CHOL_LL  left-looking: update the current block row from the finished rows
//            above (A11 -= A01^T A01, A12 -= A01^T A02), factor A11, solve A12.
//   CHOL_BD  bordered: solve the column above the diagonal A01 := X00^{-T} A01,
//            update A11 -= A01^T A01, factor A11.
enum { CHOL_RL = 0, CHOL_LL = 1, CHOL_BD = 2, CHOL_NVAR = 3 };

template <class T, int TB, int ENG, int NW, class VA>
TLA_DI void chol_diag(const VA& A, const Ctx<T>& cx, int K) {
  Tile<T, TB> c;
  tload(c, A.sub(K * TB, K * TB));
  tile_potf2<T, TB>(c, cx.wbuf, cx.n - K * TB, K * TB, cx.info);
  tstore(c, A.sub(K * TB, K * TB));
}

template <class T, int TB, int ENG, int NW, int VAR, class VA>
TLA_DI void potrf_blocked(const VA& A, const Ctx<T>& cx) {
  const int w = wave_id(), nt = cx.nt;
  typedef Gemm<T, TB, ENG> G;
  if constexpr (VAR == CHOL_RL) {
    for (int K = 0; K < nt; ++K) {
      if (w == 0) chol_diag<T, TB, ENG, NW>(A, cx, K);
      __syncthreads();
      for (int J = K + 1 + w; J < nt; J += NW) {
        Tile<T, TB> c;
        tload(c, A.sub(K * TB, J * TB));
        tile_trsm_ut<T, TB>(c, A.sub(K * TB, K * TB), cx.wbuf);
        tstore(c, A.sub(K * TB, J * TB));
      }
      __syncthreads();
      const int m = nt - K - 1;
      for (int t = w; t < m * (m + 1) / 2; t += NW) {
        int I = 0, tt = t;
        while (tt >= m - I) { tt -= m - I; ++I; }
        const int Ig = K + 1 + I, Jg = Ig + tt;
        Tile<T, TB> c;
        tload(c, A.sub(Ig * TB, Jg * TB));
        G::sub(c, A.sub(K * TB, Ig * TB).t(), A.sub(K * TB, Jg * TB));
        tstore(c, A.sub(Ig * TB, Jg * TB));
      }
      __syncthreads();
    }
  } else if constexpr (VAR == CHOL_LL) {
    for (int K = 0; K < nt; ++K) {
      // block row K: A_KJ -= sum_{P<K} A_PK^T A_PJ for J >= K; the diagonal
      // tile is factored by the wave that updated it
      for (int J = K + w; J < nt; J += NW) {
        Tile<T, TB> c;
        tload(c, A.sub(K * TB, J * TB));
        gemm_sum<G>(c, 0, K, [&](int P) { return A.sub(P * TB, K * TB).t(); }, [&](int P) { return A.sub(P * TB, J * TB); });
        if (J == K) tile_potf2<T, TB>(c, cx.wbuf, cx.n - K * TB, K * TB, cx.info);
        tstore(c, A.sub(K * TB, J * TB));
      }
      __syncthreads();
      for (int J = K + 1 + w; J < nt; J += NW) {
        Tile<T, TB> c;
        tload(c, A.sub(K * TB, J * TB));
        tile_trsm_ut<T, TB>(c, A.sub(K * TB, K * TB), cx.wbuf);
        tstore(c, A.sub(K * TB, J * TB));
      }
      __syncthreads();
    }
  } else {  // CHOL_BD
    for (int K = 0; K < nt; ++K) {
      // column above the diagonal: A_IK := X_II^{-T}(A_IK - sum_{P<I} X_PI^T A_PK),
      // a block forward substitution down the column (one wave), then
      // A_KK -= sum_{P<K} A_PK^T A_PK and factor.
      if (w == 0) {
        for (int I = 0; I < K; ++I) {
          Tile<T, TB> c;
          tload(c, A.sub(I * TB, K * TB));
          gemm_sum<G>(c, 0, I, [&](int P) { return A.sub(P * TB, I * TB).t(); }, [&](int P) { return A.sub(P * TB, K * TB); });
          tile_trsm_ut<T, TB>(c, A.sub(I * TB, I * TB), cx.wbuf);
          tstore(c, A.sub(I * TB, K * TB));
        }
        Tile<T, TB> c;
        tload(c, A.sub(K * TB, K * TB));
        gemm_sum<G>(c, 0, K, [&](int P) { return A.sub(P * TB, K * TB).t(); }, [&](int P) { return A.sub(P * TB, K * TB); });
        tile_potf2<T, TB>(c, cx.wbuf, cx.n - K * TB, K * TB, cx.info);
        tstore(c, A.sub(K * TB, K * TB));
      }
      __syncthreads();
    }
  }
}

// ================================================ Sylvester L X + X U = C
// X_IJ depends on X_KJ (K < I) through L and on X_IK (K < J) through U.
// One-dimensional partitions (X split by block rows or block columns):
//   SYL_WF  tile wavefront: all tiles with I + J = d at once, lazy updates.
//   SYL_RL  block rows, lazy:  C_I -= L_{I,<I} X_{<I}; sweep the row block.
//   SYL_RE  block rows, eager: sweep the row block; C_{>I} -= L_{>I,I} X_I.
//   SYL_CL  block columns, lazy:  C_J -= X_{<J} U_{<J,J}; sweep the column.
//   SYL_CE  block columns, eager: sweep the column; C_{>J} -= X_J U_{J,>J}.
// Two-dimensional partition.  With X, C split into quadrants TL, TR, BL, BR
// (L lower and U upper split conformally) the partitioned equation reads
//   TL:  L_TL X_TL + X_TL U_TL = C_TL
//   TR:  L_TL X_TR + X_TR U_BR = C_TR - X_TL U_TR
//   BL:  L_BR X_BL + X_BL U_TL = C_BL - L_BL X_TL
//   BR:  L_BR X_BR + X_BR U_BR = C_BR - L_BL X_TR - X_BL U_TR.
// A loop that grows TL by one block row and column per step keeps one of
// these states between steps, and each gives a variant:
//   SYL_BD  only X_TL is solved: the step solves the new column above the
//           diagonal and the new row left of it (independent of each other,
//           two waves), then the diagonal tile ("bordered").
//   SYL_BL  X_TL, X_TR and X_BL are solved, BR still holds C: the step solves
//           the diagonal tile, then the rest of its block row (one wave) and
//           of its block column (another wave), lazily.
//   SYL_BE  as SYL_BL with BR kept updated (C_BR - L_BL X_TR - X_BL U_TR):
//           after the row and column, C_{>K,>K} -= L_{>K,K} X_{K,>K} +
//           X_{>K,K} U_{K,>K} over all waves (right-looking).
// The states in which only one of TR and BL is solved give back the block
// row and block column variants above.
enum { SYL_WF = 0, SYL_RL = 1, SYL_RE = 2, SYL_CL = 3, SYL_CE = 4, SYL_BD = 5, SYL_BL = 6, SYL_BE = 7, SYL_NVAR = 8 };

// Diagonal-tile coefficients of tile (I, J) (L_II and U_JJ), fetched before
// the tile's updates so that their loads overlap the products.
template <class T, int TB, class VL, class VU>
TLA_DI auto syl_tile_fetch(const VL& L, const VU& U, int I, int J) {
  return sylv_fetch<T, TB>(L.sub(I * TB, I * TB), U.sub(J * TB, J * TB));
}
template <class T, int TB, class K>
TLA_DI void syl_tile_solve_k(Tile<T, TB>& c, const K& k, const Ctx<T>& cx, int I, int J) {
  sylv_solve<T, TB>(c, k, cx.wbuf, cx.n - I * TB, cx.n - J * TB);
}
template <class T, int TB, class VL, class VU>
TLA_DI void syl_tile_solve(Tile<T, TB>& c, const VL& L, const VU& U, const Ctx<T>& cx, int I, int J) {
  syl_tile_solve_k<T, TB>(c, syl_tile_fetch<T, TB>(L, U, I, J), cx, I, J);
}

template <class T, int TB, int ENG, int NW, int VAR, class VX, class VL, class VU>
TLA_DI void trsyl_blocked(const VX& X, const VL& L, const VU& U, const Ctx<T>& cx) {
  const int w = wave_id(), nt = cx.nt;
  typedef Gemm<T, TB, ENG> G;
  if constexpr (VAR == SYL_WF) {
    for (int d = 0; d <= 2 * nt - 2; ++d) {
      const int lo = d - nt + 1 > 0 ? d - nt + 1 : 0;
      const int hi = d < nt - 1 ? d : nt - 1;
      for (int I = lo + w; I <= hi; I += NW) {
        const int J = d - I;
        const auto k = syl_tile_fetch<T, TB>(L, U, I, J);
        Tile<T, TB> c;
        tload(c, X.sub(I * TB, J * TB));
        gemm_sum<G>(c, 0, I, [&](int K) { return L.sub(I * TB, K * TB); }, [&](int K) { return X.sub(K * TB, J * TB); });
        gemm_sum<G>(c, 0, J, [&](int K) { return X.sub(I * TB, K * TB); }, [&](int K) { return U.sub(K * TB, J * TB); });
        syl_tile_solve_k<T, TB>(c, k, cx, I, J);
        tstore(c, X.sub(I * TB, J * TB));
      }
      __syncthreads();
    }
  } else if constexpr (VAR == SYL_RL || VAR == SYL_RE) {
    for (int I = 0; I < nt; ++I) {
      if constexpr (VAR == SYL_RL) {
        for (int J = w; J < nt; J += NW) {
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, J * TB));
          gemm_sum<G>(c, 0, I, [&](int K) { return L.sub(I * TB, K * TB); }, [&](int K) { return X.sub(K * TB, J * TB); });
          tstore(c, X.sub(I * TB, J * TB));
        }
        __syncthreads();
      }
      if (w == 0) {
        for (int J = 0; J < nt; ++J) {
          const auto k = syl_tile_fetch<T, TB>(L, U, I, J);
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, J * TB));
          gemm_sum<G>(c, 0, J, [&](int K) { return X.sub(I * TB, K * TB); }, [&](int K) { return U.sub(K * TB, J * TB); });
          syl_tile_solve_k<T, TB>(c, k, cx, I, J);
          tstore(c, X.sub(I * TB, J * TB));
        }
      }
      __syncthreads();
      if constexpr (VAR == SYL_RE) {
        const int m = nt - I - 1;
        for (int t = w; t < m * nt; t += NW) {
          const int I2 = I + 1 + t / nt, J = t % nt;
          Tile<T, TB> c;
          tload(c, X.sub(I2 * TB, J * TB));
          G::sub(c, L.sub(I2 * TB, I * TB), X.sub(I * TB, J * TB));
          tstore(c, X.sub(I2 * TB, J * TB));
        }
        __syncthreads();
      }
    }
  } else if constexpr (VAR == SYL_BD) {
    const int wr = NW > 1 ? 1 : 0;
    for (int K = 0; K < nt; ++K) {
      // the finished part of every border tile's update, spread over the waves:
      // column tiles (I, K), I < K, take X_{I,<K} U_{<K,K}; row tiles (K, J),
      // J < K, take L_{K,<K} X_{<K,J}
      for (int t = w; t < 2 * K; t += NW) {
        const bool col = t < K;
        const int I = col ? t : K, J = col ? K : t - K;
        Tile<T, TB> c;
        tload(c, X.sub(I * TB, J * TB));
        if (col) gemm_sum<G>(c, 0, K, [&](int P) { return X.sub(I * TB, P * TB); }, [&](int P) { return U.sub(P * TB, K * TB); });
        else gemm_sum<G>(c, 0, K, [&](int P) { return L.sub(K * TB, P * TB); }, [&](int P) { return X.sub(P * TB, J * TB); });
        tstore(c, X.sub(I * TB, J * TB));
      }
      __syncthreads();
      // column above the diagonal, downwards (one wave) and row left of it,
      // rightwards (another wave)
      if (w == 0) {
        for (int I = 0; I < K; ++I) {
          const auto k = syl_tile_fetch<T, TB>(L, U, I, K);
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, K * TB));
          gemm_sum<G>(c, 0, I, [&](int P) { return L.sub(I * TB, P * TB); }, [&](int P) { return X.sub(P * TB, K * TB); });
          syl_tile_solve_k<T, TB>(c, k, cx, I, K);
          tstore(c, X.sub(I * TB, K * TB));
        }
      }
      if (w == wr) {
        for (int J = 0; J < K; ++J) {
          const auto k = syl_tile_fetch<T, TB>(L, U, K, J);
          Tile<T, TB> c;
          tload(c, X.sub(K * TB, J * TB));
          gemm_sum<G>(c, 0, J, [&](int P) { return X.sub(K * TB, P * TB); }, [&](int P) { return U.sub(P * TB, J * TB); });
          syl_tile_solve_k<T, TB>(c, k, cx, K, J);
          tstore(c, X.sub(K * TB, J * TB));
        }
      }
      __syncthreads();
      if (w == 0) {
        const auto k = syl_tile_fetch<T, TB>(L, U, K, K);
        Tile<T, TB> c;
        tload(c, X.sub(K * TB, K * TB));
        gemm_sum<G>(c, 0, K, [&](int P) { return L.sub(K * TB, P * TB); }, [&](int P) { return X.sub(P * TB, K * TB); });
        gemm_sum<G>(c, 0, K, [&](int P) { return X.sub(K * TB, P * TB); }, [&](int P) { return U.sub(P * TB, K * TB); });
        syl_tile_solve_k<T, TB>(c, k, cx, K, K);
        tstore(c, X.sub(K * TB, K * TB));
      }
      __syncthreads();
    }
  } else if constexpr (VAR == SYL_BL) {
    const int wr = NW > 1 ? 1 : 0;
    for (int K = 0; K < nt; ++K) {
      // finished part of the border's updates; task 0 is the diagonal tile,
      // whose update is complete, so its wave solves it at once
      const int m = nt - K - 1;
      for (int t = w; t < 2 * m + 1; t += NW) {
        const int I = t <= m ? K : K + t - m, J = t <= m ? K + t : K;
        Tile<T, TB> c;
        tload(c, X.sub(I * TB, J * TB));
        gemm_sum<G>(c, 0, K, [&](int P) { return L.sub(I * TB, P * TB); }, [&](int P) { return X.sub(P * TB, J * TB); });
        gemm_sum<G>(c, 0, K, [&](int P) { return X.sub(I * TB, P * TB); }, [&](int P) { return U.sub(P * TB, J * TB); });
        if (t == 0) syl_tile_solve<T, TB>(c, L, U, cx, K, K);
        tstore(c, X.sub(I * TB, J * TB));
      }
      __syncthreads();
      if (w == 0) {
        for (int J = K + 1; J < nt; ++J) {
          const auto k = syl_tile_fetch<T, TB>(L, U, K, J);
          Tile<T, TB> c;
          tload(c, X.sub(K * TB, J * TB));
          gemm_sum<G>(c, K, J, [&](int P) { return X.sub(K * TB, P * TB); }, [&](int P) { return U.sub(P * TB, J * TB); });
          syl_tile_solve_k<T, TB>(c, k, cx, K, J);
          tstore(c, X.sub(K * TB, J * TB));
        }
      }
      if (w == wr) {
        for (int I = K + 1; I < nt; ++I) {
          const auto k = syl_tile_fetch<T, TB>(L, U, I, K);
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, K * TB));
          gemm_sum<G>(c, K, I, [&](int P) { return L.sub(I * TB, P * TB); }, [&](int P) { return X.sub(P * TB, K * TB); });
          syl_tile_solve_k<T, TB>(c, k, cx, I, K);
          tstore(c, X.sub(I * TB, K * TB));
        }
      }
      __syncthreads();
    }
  } else if constexpr (VAR == SYL_BE) {
    const int wr = NW > 1 ? 1 : 0;
    if (w == 0) {
      Tile<T, TB> c;
      tload(c, X.sub(0, 0));
      syl_tile_solve<T, TB>(c, L, U, cx, 0, 0);
      tstore(c, X.sub(0, 0));
    }
    __syncthreads();
    for (int K = 0; K < nt; ++K) {
      // row and column of the border; only updates from inside the border remain
      if (w == 0) {
        for (int J = K + 1; J < nt; ++J) {
          const auto k = syl_tile_fetch<T, TB>(L, U, K, J);
          Tile<T, TB> c;
          tload(c, X.sub(K * TB, J * TB));
          gemm_sum<G>(c, K, J, [&](int P) { return X.sub(K * TB, P * TB); }, [&](int P) { return U.sub(P * TB, J * TB); });
          syl_tile_solve_k<T, TB>(c, k, cx, K, J);
          tstore(c, X.sub(K * TB, J * TB));
        }
      }
      if (w == wr) {
        for (int I = K + 1; I < nt; ++I) {
          const auto k = syl_tile_fetch<T, TB>(L, U, I, K);
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, K * TB));
          gemm_sum<G>(c, K, I, [&](int P) { return L.sub(I * TB, P * TB); }, [&](int P) { return X.sub(P * TB, K * TB); });
          syl_tile_solve_k<T, TB>(c, k, cx, I, K);
          tstore(c, X.sub(I * TB, K * TB));
        }
      }
      __syncthreads();
      // trailing update C_IJ -= L_IK X_KJ + X_IK U_KJ for I, J > K; task 0 is
      // the next diagonal tile, which its wave then solves
      const int m = nt - K - 1;
      for (int t = w; t < m * m; t += NW) {
        const int I = K + 1 + t / m, J = K + 1 + t % m;
        Tile<T, TB> c;
        tload(c, X.sub(I * TB, J * TB));
        G::sub(c, L.sub(I * TB, K * TB), X.sub(K * TB, J * TB));
        G::sub(c, X.sub(I * TB, K * TB), U.sub(K * TB, J * TB));
        if (t == 0) syl_tile_solve<T, TB>(c, L, U, cx, I, J);
        tstore(c, X.sub(I * TB, J * TB));
      }
      __syncthreads();
    }
  } else {  // SYL_CL / SYL_CE
    for (int J = 0; J < nt; ++J) {
      if constexpr (VAR == SYL_CL) {
        for (int I = w; I < nt; I += NW) {
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, J * TB));
          gemm_sum<G>(c, 0, J, [&](int K) { return X.sub(I * TB, K * TB); }, [&](int K) { return U.sub(K * TB, J * TB); });
          tstore(c, X.sub(I * TB, J * TB));
        }
        __syncthreads();
      }
      if (w == 0) {
        for (int I = 0; I < nt; ++I) {
          const auto k = syl_tile_fetch<T, TB>(L, U, I, J);
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, J * TB));
          gemm_sum<G>(c, 0, I, [&](int K) { return L.sub(I * TB, K * TB); }, [&](int K) { return X.sub(K * TB, J * TB); });
          syl_tile_solve_k<T, TB>(c, k, cx, I, J);
          tstore(c, X.sub(I * TB, J * TB));
        }
      }
      __syncthreads();
      if constexpr (VAR == SYL_CE) {
        const int m = nt - J - 1;
        for (int t = w; t < m * nt; t += NW) {
          const int J2 = J + 1 + t / nt, I = t % nt;
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, J2 * TB));
          G::sub(c, X.sub(I * TB, J * TB), U.sub(J * TB, J2 * TB));
          tstore(c, X.sub(I * TB, J2 * TB));
        }
        __syncthreads();
      }
    }
  }
}

// =============================================== Lyapunov L X + X L^T = S
// Only the lower tiles I >= J are computed (X symmetric).  Tile (I, J) obeys
//   L_II X_IJ + X_IJ L_JJ^T = S_IJ - sum_{K<I} L_IK X_KJ - sum_{K<J} X_IK L_JK^T
// with X_KJ = X_JK^T for K < J; diagonal tiles are Lyapunov tiles, solved as
// Sylvester tiles with U = L_II^T and then made exactly symmetric from their
// lower triangle.
//   LYA_WF  tile wavefront over the lower tiles, lazy updates.
//   LYA_RL  block rows, lazy: column-side updates of the whole block row at
//           once, then a sweep along the row.
//   LYA_RE  right-looking (eager) by block column: diagonal tile, the tiles
//           below it, then the symmetric rank-2b update of the trailing part.
//   LYA_CL  block columns, lazy: the updates from the finished columns for the
//           whole block column at once (the diagonal tile is then complete and
//           solved), then a sweep down the column.
// With X symmetric the two-dimensional partition of the Sylvester case folds
// onto the lower triangle: its "bordered" state is LYA_RL, the lazy and eager
// border states are LYA_CL and LYA_RE.
enum { LYA_WF = 0, LYA_RL = 1, LYA_RE = 2, LYA_CL = 3, LYA_NVAR = 4 };

template <class T, int TB, class VL>
TLA_DI auto lya_tile_fetch(const VL& L, int I, int J) {
  return sylv_fetch<T, TB>(L.sub(I * TB, I * TB), L.sub(J * TB, J * TB).t());
}
template <class T, int TB, class VX, class K>
TLA_DI void lya_tile_solve_k(Tile<T, TB>& c, const VX& X, const K& k, const Ctx<T>& cx, int I, int J) {
  sylv_solve<T, TB>(c, k, cx.wbuf, cx.n - I * TB, cx.n - J * TB);
  if (I == J) {
    // store the lower triangle into both halves: the tile becomes exactly symmetric
    const int l = lane_id(), j = tcol<TB>(l);
#pragma unroll
    for (int r = 0; r < Tile<T, TB>::EPL; ++r) {
      const int i = trow<T, TB>(l, r);
      if (i >= j) {
        X.store(I * TB + i, J * TB + j, c.v[r]);
        X.store(J * TB + j, I * TB + i, c.v[r]);
      }
    }
    X.fence();
  } else {
    tstore(c, X.sub(I * TB, J * TB));
    if constexpr (VX::mirrors()) tstore(c, X.sub(J * TB, I * TB).t());
  }
}
template <class T, int TB, class VX, class VL>
TLA_DI void lya_tile_solve(Tile<T, TB>& c, const VX& X, const VL& L, const Ctx<T>& cx, int I, int J) {
  lya_tile_solve_k<T, TB>(c, X, lya_tile_fetch<T, TB>(L, I, J), cx, I, J);
}

// column-side lazy update: c -= sum_{K in [k0,k1)} L_IK X~_KJ, X~_KJ = X_KJ (K >= J) or X_JK^T
template <class T, int TB, int ENG, class VX, class VL>
TLA_DI void lya_colside(Tile<T, TB>& c, const VX& X, const VL& L, int I, int J, int k0, int k1) {
  typedef Gemm<T, TB, ENG> G;
  gemm_sum<G>(c, k0, k1, [&](int K) { return L.sub(I * TB, K * TB); },
              [&](int K) { return K >= J ? X.sub(K * TB, J * TB) : X.sub(J * TB, K * TB).t(); });
}
// row-side lazy update: c -= sum_{K in [k0,k1)} X_IK L_JK^T
template <class T, int TB, int ENG, class VX, class VL>
TLA_DI void lya_rowside(Tile<T, TB>& c, const VX& X, const VL& L, int I, int J, int k0, int k1) {
  typedef Gemm<T, TB, ENG> G;
  gemm_sum<G>(c, k0, k1, [&](int K) { return X.sub(I * TB, K * TB); }, [&](int K) { return L.sub(J * TB, K * TB).t(); });
}

template <class T, int TB, int ENG, int NW, int VAR, class VX, class VL>
TLA_DI void trlyap_blocked(const VX& X, const VL& L, const Ctx<T>& cx) {
  const int w = wave_id(), nt = cx.nt;
  typedef Gemm<T, TB, ENG> G;
  if constexpr (VAR == LYA_WF) {
    for (int d = 0; d <= 2 * nt - 2; ++d) {
      const int lo = (d + 1) / 2;
      const int hi = d < nt - 1 ? d : nt - 1;
      for (int I = lo + w; I <= hi; I += NW) {
        const int J = d - I;
        const auto k = lya_tile_fetch<T, TB>(L, I, J);
        Tile<T, TB> c;
        tload(c, X.sub(I * TB, J * TB));
        lya_colside<T, TB, ENG>(c, X, L, I, J, 0, I);
        lya_rowside<T, TB, ENG>(c, X, L, I, J, 0, J);
        lya_tile_solve_k<T, TB>(c, X, k, cx, I, J);
      }
      __syncthreads();
    }
  } else if constexpr (VAR == LYA_RL) {
    for (int I = 0; I < nt; ++I) {
      // off-diagonal tiles of the row only: the diagonal tile's column-side
      // term sum_{K<I} L_IK X_IK^T needs this row's own results
      for (int J = w; J < I; J += NW) {
        Tile<T, TB> c;
        tload(c, X.sub(I * TB, J * TB));
        lya_colside<T, TB, ENG>(c, X, L, I, J, 0, I);
        tstore(c, X.sub(I * TB, J * TB));
      }
      __syncthreads();
      if (w == 0) {
        for (int J = 0; J <= I; ++J) {
          const auto k = lya_tile_fetch<T, TB>(L, I, J);
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, J * TB));
          if (J == I) lya_colside<T, TB, ENG>(c, X, L, I, J, 0, I);
          lya_rowside<T, TB, ENG>(c, X, L, I, J, 0, J);
          lya_tile_solve_k<T, TB>(c, X, k, cx, I, J);
        }
      }
      __syncthreads();
    }
  } else if constexpr (VAR == LYA_CL) {
    for (int J = 0; J < nt; ++J) {
      // tiles (I, J), I >= J: the terms through the finished columns K < J,
      // sum_{K<J} L_IK X_JK^T + X_IK L_JK^T; task 0 is the diagonal tile
      for (int I = J + w; I < nt; I += NW) {
        Tile<T, TB> c;
        tload(c, X.sub(I * TB, J * TB));
        lya_colside<T, TB, ENG>(c, X, L, I, J, 0, J);
        lya_rowside<T, TB, ENG>(c, X, L, I, J, 0, J);
        if (I == J) lya_tile_solve<T, TB>(c, X, L, cx, J, J);
        else tstore(c, X.sub(I * TB, J * TB));
      }
      __syncthreads();
      // down the column: the remaining terms sum_{J<=K<I} L_IK X_KJ
      if (w == 0) {
        for (int I = J + 1; I < nt; ++I) {
          const auto k = lya_tile_fetch<T, TB>(L, I, J);
          Tile<T, TB> c;
          tload(c, X.sub(I * TB, J * TB));
          lya_colside<T, TB, ENG>(c, X, L, I, J, J, I);
          lya_tile_solve_k<T, TB>(c, X, k, cx, I, J);
        }
      }
      __syncthreads();
    }
  } else {  // LYA_RE
    for (int K = 0; K < nt; ++K) {
      if (w == 0) {
        Tile<T, TB> c;
        tload(c, X.sub(K * TB, K * TB));
        lya_tile_solve<T, TB>(c, X, L, cx, K, K);
        // tiles below: L_II X_IK + X_IK L_KK^T = S_IK - L_IK X_KK - sum_{K<P<I} L_IP X_PK
        for (int I = K + 1; I < nt; ++I) {
          const auto k = lya_tile_fetch<T, TB>(L, I, K);
          tload(c, X.sub(I * TB, K * TB));
          gemm_sum<G>(c, K, I, [&](int P) { return L.sub(I * TB, P * TB); }, [&](int P) { return X.sub(P * TB, K * TB); });
          lya_tile_solve_k<T, TB>(c, X, k, cx, I, K);
        }
      }
      __syncthreads();
      // trailing: S_IJ -= L_IK X_JK^T + X_IK L_JK^T for I >= J > K
      const int m = nt - K - 1;
      for (int t = w; t < m * (m + 1) / 2; t += NW) {
        int jj = 0, tt = t;
        while (tt >= m - jj) { tt -= m - jj; ++jj; }
        const int J = K + 1 + jj, I = J + tt;
        Tile<T, TB> c;
        tload(c, X.sub(I * TB, J * TB));
        G::sub(c, L.sub(I * TB, K * TB), X.sub(J * TB, K * TB).t());
        G::sub(c, X.sub(I * TB, K * TB), L.sub(J * TB, K * TB).t());
        tstore(c, X.sub(I * TB, J * TB));
      }
      __syncthreads();
    }
  }
}

}  // namespace tla
