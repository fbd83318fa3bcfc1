// Mixed precision with FP64 refinement, one workgroup per instance.
//
// The paper computes in double precision only.  Here each instance is
// first solved in FP32 (tile updates on the FP32, FP16 or BF16 matrix cores
// with FP32 accumulation, diagonal tiles in FP32 vector arithmetic), then
// refined in FP64 until the backward error eta drops below tau:
//   Sylvester / Lyapunov (classical refinement):
//     R = C - (L X + X U) in FP64, eta, D = solve_lo(R), X += D in FP64.
//   Cholesky (Newton correction of the factor): with R = A - X^T X,
//     linearising (X+E)^T (X+E) = A gives X^T E + E^T X = R; E = F X with F
//     upper triangular solves it when F + F^T = X^{-T} R X^{-1} = M, so
//     F = triu(M) with its diagonal halved and X += F X.
// Only the residual, the correction accumulation and the fallback run in
// FP64.  Refinement stops with FALLBACK when eta_k > eta_{k-1}/2 (stall) or
// after max_iter corrections, with BREAKDOWN when the low-precision solve
// meets a zero pivot/denominator or produces a non-finite value; both then
// solve the instance again by the FP64 kernel code.  Input and output are
// FP64; the FP64 solution lives in LDS (Xd) next to the FP32 work matrix (W).
#pragma once
#include "tla_kernels.hpp"

namespace tla {

template <int NW>
TLA_DI double block_sum(double v, double* red) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < NW; ++w) s += red[w];
  return s;
}

template <int NW>
TLA_DI int block_or(int v, int* red) {
  __syncthreads();
  if (threadIdx.x == 0) *red = 0;
  __syncthreads();
  if (v) atomicOr(red, v);
  __syncthreads();
  return *red;
}

// Which FP64 tile engine the residual and the fallback use.
template <int TB>
struct F64Eng { static constexpr int value = TB == 16 ? ENG_MFMA : ENG_VALU; };

// Convergence bookkeeping shared by the three operations.
struct RefineState {
  double eta, prev;
  int it, flags;
};

// Decide after a residual: returns true when the loop must stop.
TLA_DI bool refine_decide(RefineState& st, double eta, double tau, int max_iter) {
  st.eta = eta;
  if (eta <= tau) { st.flags |= TLA_STAT_CONVERGED; return true; }
  if (!(eta == eta) || st.it >= max_iter || !(eta <= 0.5 * st.prev)) { st.flags |= TLA_STAT_FALLBACK; return true; }
  st.prev = eta;
  return false;
}

TLA_DI void write_stat(const Inst& in, const RefineState& st) {
  if (threadIdx.x == 0 && in.stat) {
    in.stat->iters = st.it;
    in.stat->flags = st.flags;
    in.stat->eta = st.eta;
  }
}

// LDS carve-up of the mixed kernels: Xd (FP64), W (FP32), aux (FP32:
// coefficients or the FP32 factor), scratch, reduction cells.
struct MixedLds {
  double* Xd;
  float* W;
  float* A1;
  float* A2;
  float* wb;
  double* red;
  int* ired;
  int* info;
};

// With XG the FP64 solution lives in a global workspace slot instead (sizes
// where it does not fit next to W), followed there by the FP32 auxiliary
// matrices; every access to them is separated by workgroup barriers, and the
// FP64 fallback runs as a second launch.  With WG
// (which implies XG) the FP32 work matrix and the FP32 auxiliary matrices
// follow it into the slot, after the solution, and LDS keeps only the tile
// solvers' scratch and the reduction cells.
template <int TB, int NW, bool XG, bool WG = false>
TLA_DI MixedLds carve(unsigned char* smem, const KArgs& g, int naux) {
  static_assert(!WG || XG, "the work matrix only leaves LDS with the solution");
  const size_t np = (size_t)g.ntmax * TB, mat = np * (np + 1);
  MixedLds m;
  float* after;
  if constexpr (WG) {
    m.Xd = g.work + (size_t)blockIdx.x * g.work_stride;
    m.W = reinterpret_cast<float*>(m.Xd + mat);
    m.A1 = m.W + mat;
    m.A2 = m.A1 + (naux >= 1 ? mat : 0);
    after = reinterpret_cast<float*>(smem);
  } else {
    if constexpr (XG) {
      // the FP32 auxiliary matrices (the Cholesky factor copy) follow the
      // solution into the workspace; LDS keeps the work matrix
      m.Xd = g.work + (size_t)blockIdx.x * g.work_stride;
      m.W = reinterpret_cast<float*>(smem);
      m.A1 = reinterpret_cast<float*>(m.Xd + mat);
      m.A2 = m.A1 + (naux >= 1 ? mat : 0);
      after = m.W + mat;
    } else {
      m.Xd = reinterpret_cast<double*>(smem);
      m.W = reinterpret_cast<float*>(m.Xd + mat);
      m.A1 = m.W + mat;
      m.A2 = m.A1 + (naux >= 1 ? mat : 0);
      after = m.A2 + (naux >= 2 ? mat : 0);
    }
  }
  // tile solvers' scratch, 8-byte aligned: FP32 elements when the FP64
  // fallback is a second launch (XG), else FP64 (the fallback solve reuses it)
  m.wb = reinterpret_cast<float*>((reinterpret_cast<uintptr_t>(after) + 7) & ~uintptr_t(7));
  m.red = reinterpret_cast<double*>(reinterpret_cast<unsigned char*>(m.wb) +
                                    (size_t)NW * wave_scratch(TB) * (XG ? sizeof(float) : sizeof(double)));
  m.ired = reinterpret_cast<int*>(m.red + NW + 1);
  m.info = m.ired + 1;
  return m;
}

// Two-wave Sylvester and Lyapunov kernels with the FP64 solution in the
// workspace fit 7 instances per compute unit in LDS; their registers are held
// to 4 resident waves per SIMD to match (the compiler alone allows 3).
template <int NW, bool XG, bool WG>
constexpr int kMixedWaves = (NW == 2 && XG && !WG) ? 4 : 1;

// True when every entry of the n x n leading block is finite (work matrix in
// LDS, or in global memory for !LDS).
template <class T, bool LDS = true>
TLA_DI bool all_finite(const T* Wg, int ldw, int n) {
  const auto W = xcolmajor<!LDS>(const_cast<T*>(Wg), ldw);
  bool ok = true;
  const int nw = blockDim.x >> 6;
  for (int j = wave_id(); j < n; j += nw)
    for (int i = lane_id(); i < n; i += 64) {
      const T v = W(i, j);
      ok = ok && (v - v == T(0));
    }
  return ok;
}

// Writes the symmetric n x n result held in the lower triangle of a global
// work matrix (leading dimension ldx) to the caller's matrix, by 16 x 16
// tiles: each tile below the diagonal is stored in place and transposed
// above it (both stores coalesced), a diagonal tile from its lower triangle.
// Reads and writes outside n x n are clamped or dropped.
template <int NW>
TLA_DI void egress_sym_tiles(double* Gg, int ldg, int n, const double* Xg, int ldx) {
  const GView<double> X = gview<double>(Xg, ldx, n, 0);
  gbl_t<double>* G = to_gbl(Gg);
  const int nt = (n + 15) / 16, l = lane_id(), j = tcol<16>(l);
  for (int t = wave_id(); t < nt * nt; t += NW) {
    const int I = t / nt, J = t - I * nt;
    if (I < J) continue;
    Tile<double, 16> c;
    tload(c, X.sub(I * 16, J * 16));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = trow<double, 16>(l, r), gi = I * 16 + i, gj = J * 16 + j;
      if (gi >= n || gj >= n || (I == J && i < j)) continue;
      G[gi + (size_t)gj * ldg] = c.v[r];
      if (gi != gj) G[gj + (size_t)gi * ldg] = c.v[r];
    }
  }
}

// ===================================================== Sylvester, mixed
template <int TB, int ENG, int NW, int VAR, bool LU_LDS, bool XG, bool WG = false>
TLA_DI void trsyl_mixed_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  static_assert(!(LU_LDS && XG), "coefficients in LDS only with the solution in LDS");
  int n;
  if (!validate(in, g.n_max, n)) return;
  const int nt = (n + TB - 1) / TB, np = nt * TB, ld = np + 1;
  const MixedLds m = carve<TB, NW, XG, WG>(smem, g, LU_LDS ? 2 : 0);
  const double* Lg = in.a;
  const double* Ug = in.b;
  double* Cg = in.c;
  const int ldl = in.lda, ldu = in.ldb, ldc = in.ldc;
  const GView<double> L64 = gview<double>(Lg, ldl, n, -1);
  const GView<double> U64 = gview<double>(Ug, ldu, n, +1);
  const GView<double> C64 = gview<double>(Cg, ldc, n, 0);
  constexpr int E64 = F64Eng<TB>::value;
  if (threadIdx.x == 0) *m.info = INT_MAX;
  RefineState st{INFINITY, INFINITY, 0, 0};

  double sc = ingest<float, NW, !WG>(m.W, ld, np, Cg, ldc, n, 0, 0.0f);
  double sl = 0.0, su = 0.0;
  if constexpr (LU_LDS) {
    sl = ingest<float, NW>(m.A1, ld, np, Lg, ldl, n, -1, 0.0f);
    su = ingest<float, NW>(m.A2, ld, np, Ug, ldu, n, +1, 0.0f);
  } else {
    sl = gnorm2<NW>(Lg, ldl, n, -1);
    su = gnorm2<NW>(Ug, ldu, n, +1);
  }
  const double nc = sqrt(block_sum<NW>(sc, m.red));
  const double nl = sqrt(block_sum<NW>(sl, m.red));
  const double nu = sqrt(block_sum<NW>(su, m.red));
  int bad = (nc - nc != 0.0 || nl - nl != 0.0 || nu - nu != 0.0) ? TLA_STAT_NONFINITE : 0;
  // exact zero denominators (FP64) decide info; FP32 ones only force the FP64 path
  const int lo_zero = scan_zero_denoms<true>(L64, U64, n, false, m.info) ? TLA_STAT_BREAKDOWN : 0;
  bad |= block_or<NW>(lo_zero | bad, m.ired);
  st.flags |= bad;
  const int info0 = *m.info == INT_MAX ? 0 : *m.info;
  Ctx<float> cx{n, nt, to_lds(m.wb + wave_id() * wave_scratch(TB)), to_lds(m.info)};
  if (info0 == 0 && !bad) {
    // low-precision solve of the full system
    if constexpr (LU_LDS) trsyl_blocked<float, TB, ENG, NW, VAR>(xcolmajor<WG>(m.W, ld), colmajor(m.A1, ld), colmajor(m.A2, ld), cx);
    else trsyl_blocked<float, TB, ENG, NW, VAR>(xcolmajor<WG>(m.W, ld), gview<float>(Lg, ldl, n, -1), gview<float>(Ug, ldu, n, +1), cx);
    __syncthreads();
    if (block_or<NW>(all_finite<float, !WG>(m.W, ld, n) ? 0 : 1, m.ired)) st.flags |= TLA_STAT_BREAKDOWN;
    if (!(st.flags & TLA_STAT_BREAKDOWN)) {
      for (int e = threadIdx.x; e < np * ld; e += blockDim.x) m.Xd[e] = double(m.W[e]);
      __syncthreads();
      for (;;) {
        // R = C - L Xd - Xd U (FP64), into W; squared norms of R and Xd
        double sr = 0.0, sx = 0.0;
        const auto Xv = xcolmajor<XG>(m.Xd, ld);
        for (int t = wave_id(); t < nt * nt; t += NW) {
          const int I = t / nt, J = t - I * nt;
          Tile<double, TB> c, x;
          tload(c, C64.sub(I * TB, J * TB));
          tload(x, Xv.sub(I * TB, J * TB));
          typedef Gemm<double, TB, E64> G64;
          gemm_sum<G64>(c, 0, I + 1, [&](int K) { return L64.sub(I * TB, K * TB); }, [&](int K) { return Xv.sub(K * TB, J * TB); });
          gemm_sum<G64>(c, 0, J + 1, [&](int K) { return Xv.sub(I * TB, K * TB); }, [&](int K) { return U64.sub(K * TB, J * TB); });
          const int l = lane_id(), j = tcol<TB>(l);
#pragma unroll
          for (int r = 0; r < Tile<double, TB>::EPL; ++r) {
            const int i = trow<double, TB>(l, r);
            m.W[(I * TB + i) + (J * TB + j) * ld] = float(c.v[r]);
            sr += c.v[r] * c.v[r];
            sx += x.v[r] * x.v[r];
          }
        }
        const double nr = sqrt(block_sum<NW>(sr, m.red));
        const double nx = sqrt(block_sum<NW>(sx, m.red));
        const double eta = nr / ((nl + nu) * nx + nc);
        if (refine_decide(st, eta, g.tau, g.max_iter)) break;
        __syncthreads();
        if constexpr (LU_LDS) trsyl_blocked<float, TB, ENG, NW, VAR>(xcolmajor<WG>(m.W, ld), colmajor(m.A1, ld), colmajor(m.A2, ld), cx);
        else trsyl_blocked<float, TB, ENG, NW, VAR>(xcolmajor<WG>(m.W, ld), gview<float>(Lg, ldl, n, -1), gview<float>(Ug, ldu, n, +1), cx);
        __syncthreads();
        for (int e = threadIdx.x; e < np * ld; e += blockDim.x) m.Xd[e] += double(m.W[e]);
        ++st.it;
        __syncthreads();
      }
    }
  }
  __syncthreads();
  const bool fb = info0 == 0 && !(st.flags & TLA_STAT_CONVERGED);
  if (!XG && fb) {
    // FP64 solve of the instance (fallback or breakdown)
    ingest<double, NW>(m.Xd, ld, np, Cg, ldc, n, 0, 0.0);
    __syncthreads();
    Ctx<double> cd{n, nt, to_lds(reinterpret_cast<double*>(m.wb) + wave_id() * wave_scratch(TB)), to_lds(m.info)};
    constexpr int ENG64 = ENG == ENG_VALU ? ENG_VALU : E64;
    trsyl_blocked<double, TB, ENG64, NW, VAR>(xcolmajor<XG>(m.Xd, ld), L64, U64, cd);
    __syncthreads();
  }
  if (info0 == 0 && !(XG && fb)) egress<double, NW, !XG>(Cg, ldc, n, m.Xd, ld, 0);
  if (threadIdx.x == 0) *in.info = info0;
  write_stat(in, st);
}

template <int TB, int ENG, int NW, int VAR, bool LU_LDS, bool XG, bool WG = false>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(kMixedWaves<NW, XG, WG>))) void k_trsyl_mixed(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  trsyl_mixed_body<TB, ENG, NW, VAR, LU_LDS, XG, WG>(g, fetch_uniform(g, blockIdx.x), smem);
}

// ===================================================== Lyapunov, mixed
template <int TB, int ENG, int NW, int VAR, bool LU_LDS, bool XG, bool WG = false>
TLA_DI void trlyap_mixed_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  static_assert(!(LU_LDS && XG), "coefficients in LDS only with the solution in LDS");
  int n;
  if (!validate(in, g.n_max, n)) return;
  const int nt = (n + TB - 1) / TB, np = nt * TB, ld = np + 1;
  const MixedLds m = carve<TB, NW, XG, WG>(smem, g, LU_LDS ? 1 : 0);
  const double* Lg = in.a;
  double* Sg = in.c;
  const int ldl = in.lda, lds = in.ldc;
  const GView<double> L64 = gview<double>(Lg, ldl, n, -1);
  const GView<double> S64 = gview<double>(Sg, lds, n, -2);
  constexpr int E64 = F64Eng<TB>::value;
  if (threadIdx.x == 0) *m.info = INT_MAX;
  RefineState st{INFINITY, INFINITY, 0, 0};

  double ss = ingest<float, NW, !WG>(m.W, ld, np, Sg, lds, n, -1, 0.0f, true);
  double sl = 0.0;
  if constexpr (LU_LDS) {
    sl = ingest<float, NW>(m.A1, ld, np, Lg, ldl, n, -1, 0.0f);
  } else {
    sl = gnorm2<NW>(Lg, ldl, n, -1);
  }
  __syncthreads();
  mirror_lower<float, !WG>(m.W, ld, np);
  const double ns = sqrt(block_sum<NW>(ss, m.red));
  const double nl = sqrt(block_sum<NW>(sl, m.red));
  int bad = (ns - ns != 0.0 || nl - nl != 0.0) ? TLA_STAT_NONFINITE : 0;
  const int lo_zero = scan_zero_denoms<true>(L64, L64, n, true, m.info) ? TLA_STAT_BREAKDOWN : 0;
  bad |= block_or<NW>(lo_zero | bad, m.ired);
  st.flags |= bad;
  const int info0 = *m.info == INT_MAX ? 0 : *m.info;
  Ctx<float> cx{n, nt, to_lds(m.wb + wave_id() * wave_scratch(TB)), to_lds(m.info)};
  if (info0 == 0 && !bad) {
    if constexpr (LU_LDS) trlyap_blocked<float, TB, ENG, NW, VAR>(xcolmajor<WG>(m.W, ld), colmajor(m.A1, ld), cx);
    else trlyap_blocked<float, TB, ENG, NW, VAR>(xcolmajor<WG>(m.W, ld), gview<float>(Lg, ldl, n, -1), cx);
    __syncthreads();
    mirror_lower<float, !WG>(m.W, ld, np);
    __syncthreads();
    if (block_or<NW>(all_finite<float, !WG>(m.W, ld, n) ? 0 : 1, m.ired)) st.flags |= TLA_STAT_BREAKDOWN;
    if (!(st.flags & TLA_STAT_BREAKDOWN)) {
      for (int e = threadIdx.x; e < np * ld; e += blockDim.x) m.Xd[e] = double(m.W[e]);
      __syncthreads();
      for (;;) {
        // R = S - L Xd - Xd L^T on the lower tiles.  Only Xd's lower tiles
        // are read (a tile above the diagonal as the transpose of its mirror),
        // and its diagonal tiles are kept exactly symmetric
        double sr = 0.0, sx = 0.0;
        const auto Xv = xcolmajor<XG>(m.Xd, ld);
        for (int t = wave_id(); t < nt * nt; t += NW) {
          const int I = t / nt, J = t - I * nt;
          if (I < J) continue;
          Tile<double, TB> c, x;
          tload(c, S64.sub(I * TB, J * TB));
          tload(x, Xv.sub(I * TB, J * TB));
          typedef Gemm<double, TB, E64> G64;
          gemm_sum<G64>(c, 0, I + 1, [&](int K) { return L64.sub(I * TB, K * TB); },
                        [&](int K) { return K >= J ? Xv.sub(K * TB, J * TB) : Xv.sub(J * TB, K * TB).t(); });
          gemm_sum<G64>(c, 0, J + 1, [&](int K) { return Xv.sub(I * TB, K * TB); }, [&](int K) { return L64.sub(J * TB, K * TB).t(); });
          const double wgt = I == J ? 1.0 : 2.0;
          const int l = lane_id(), j = tcol<TB>(l);
#pragma unroll
          for (int r = 0; r < Tile<double, TB>::EPL; ++r) {
            const int i = trow<double, TB>(l, r);
            m.W[(I * TB + i) + (J * TB + j) * ld] = float(c.v[r]);
            sr += wgt * c.v[r] * c.v[r];
            sx += wgt * x.v[r] * x.v[r];
          }
        }
        const double nr = sqrt(block_sum<NW>(sr, m.red));
        const double nx = sqrt(block_sum<NW>(sx, m.red));
        const double eta = nr / (2.0 * nl * nx + ns);
        if (refine_decide(st, eta, g.tau, g.max_iter)) break;
        __syncthreads();
        if constexpr (LU_LDS) trlyap_blocked<float, TB, ENG, NW, VAR>(xcolmajor<WG>(m.W, ld), colmajor(m.A1, ld), cx);
        else trlyap_blocked<float, TB, ENG, NW, VAR>(xcolmajor<WG>(m.W, ld), gview<float>(Lg, ldl, n, -1), cx);
        __syncthreads();
        // Xd += D on the lower tiles and on both halves of the diagonal tiles
        // (D's diagonal tiles are exactly symmetric, so Xd's stay so)
        for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
          const int j = e / np, i = e - j * np;
          if (i >= j || i / TB == j / TB) m.Xd[i + j * ld] += double(m.W[i + j * ld]);
        }
        ++st.it;
        __syncthreads();
      }
    }
  }
  __syncthreads();
  const bool fb = info0 == 0 && !(st.flags & TLA_STAT_CONVERGED);
  if (!XG && fb) {
    ingest<double, NW>(m.Xd, ld, np, Sg, lds, n, -1, 0.0);
    __syncthreads();
    mirror_lower<double, !XG>(m.Xd, ld, np);
    __syncthreads();
    Ctx<double> cd{n, nt, to_lds(reinterpret_cast<double*>(m.wb) + wave_id() * wave_scratch(TB)), to_lds(m.info)};
    constexpr int ENG64 = ENG == ENG_VALU ? ENG_VALU : E64;
    trlyap_blocked<double, TB, ENG64, NW, VAR>(xcolmajor<XG>(m.Xd, ld), L64, cd);
    __syncthreads();
  }
  if (info0 == 0 && !(XG && fb)) {
    if constexpr (XG) egress_sym_tiles<NW>(Sg, lds, n, m.Xd, ld);
    else egress<double, NW, true>(Sg, lds, n, m.Xd, ld, 2);
  }
  if (threadIdx.x == 0) *in.info = info0;
  write_stat(in, st);
}

template <int TB, int ENG, int NW, int VAR, bool LU_LDS, bool XG, bool WG = false>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(kMixedWaves<NW, XG, WG>))) void k_trlyap_mixed(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  trlyap_mixed_body<TB, ENG, NW, VAR, LU_LDS, XG, WG>(g, fetch_uniform(g, blockIdx.x), smem);
}

// ====================================================== Cholesky, mixed
// Tile solves of the Newton correction, FP32 (X32 upper factor in aux):
//   M1 = X^{-T} R   column tile by column tile (forward substitution down)
//   M  = M1 X^{-1}  row tile by row tile (substitution to the right)
template <class T, int TB, int ENG, int NW, class VW, class VF, class VXd>
TLA_DI void newton_correction(const VW& Wv, const VF& Xv, const VXd& Xd, int nt, lds_t<T>* wbuf) {
  typedef Gemm<T, TB, ENG> G;
  const int w = wave_id();
  for (int J = w; J < nt; J += NW) {
    for (int I = 0; I < nt; ++I) {
      Tile<T, TB> c;
      tload(c, Wv.sub(I * TB, J * TB));
      gemm_sum<G>(c, 0, I, [&](int K) { return Xv.sub(K * TB, I * TB).t(); }, [&](int K) { return Wv.sub(K * TB, J * TB); });
      tile_trsm_ut<T, TB>(c, Xv.sub(I * TB, I * TB), wbuf);
      tstore(c, Wv.sub(I * TB, J * TB));
    }
  }
  __syncthreads();
  for (int I = w; I < nt; I += NW) {
    for (int J = 0; J < nt; ++J) {
      Tile<T, TB> c;
      tload(c, Wv.sub(I * TB, J * TB));
      gemm_sum<G>(c, 0, J, [&](int K) { return Wv.sub(I * TB, K * TB); }, [&](int K) { return Xv.sub(K * TB, J * TB); });
      tile_trsm_right_u<T, TB>(c, Xv.sub(J * TB, J * TB), wbuf);
      tstore(c, Wv.sub(I * TB, J * TB));
    }
  }
  __syncthreads();
  // F = triu(M), diagonal halved (in place on the diagonal tiles' elements)
  for (int e = threadIdx.x; e < nt * TB * nt * TB; e += blockDim.x) {
    const int np = nt * TB;
    const int j = e / np, i = e - j * np;
    if (i > j) Wv.at(i, j) = T(0);
    else if (i == j) Wv.at(i, j) = T(0.5) * Wv(i, j);
  }
  __syncthreads();
  // E = F X on the upper tiles; Xd += E
  for (int t = w; t < nt * nt; t += NW) {
    const int I = t / nt, J = t - I * nt;
    if (I > J) continue;
    Tile<T, TB> c;
    tzero(c);
    gemm_sum<G>(c, I, J + 1, [&](int K) { return Wv.sub(I * TB, K * TB); }, [&](int K) { return Xv.sub(K * TB, J * TB); });
    const int l = lane_id(), j = tcol<TB>(l);
#pragma unroll
    for (int r = 0; r < Tile<T, TB>::EPL; ++r) {
      const int i = trow<T, TB>(l, r);
      if (I * TB + i <= J * TB + j) Xd.store(I * TB + i, J * TB + j, Xd(I * TB + i, J * TB + j) - double(c.v[r]));  // c holds -E
    }
  }
}

template <int TB, int ENG, int NW, int VAR, bool XG, bool WG = false>
TLA_DI void potrf_mixed_body(const KArgs& g, const Inst& in, unsigned char* smem) {
  int n;
  if (!validate(in, g.n_max, n)) return;
  const int nt = (n + TB - 1) / TB, np = nt * TB, ld = np + 1;
  const MixedLds m = carve<TB, NW, XG, WG>(smem, g, 1);
  double* Ag = in.c;
  const int lda = in.ldc;
  const GView<double> A64 = gview<double>(Ag, lda, n, 2);
  constexpr int E64 = F64Eng<TB>::value;
  if (threadIdx.x == 0) *m.info = 0;
  RefineState st{INFINITY, INFINITY, 0, 0};

  const double na = sqrt(block_sum<NW>(ingest<float, NW, !WG>(m.W, ld, np, Ag, lda, n, +1, 1.0f, true), m.red));
  int bad = (na - na != 0.0) ? TLA_STAT_NONFINITE : 0;
  Ctx<float> cx{n, nt, to_lds(m.wb + wave_id() * wave_scratch(TB)), to_lds(m.info)};
  if (!bad) {
    potrf_blocked<float, TB, ENG, NW, VAR>(xcolmajor<WG>(m.W, ld), cx);
    __syncthreads();
    if (*m.info != 0 || block_or<NW>(all_finite<float, !WG>(m.W, ld, n) ? 0 : 1, m.ired)) bad |= TLA_STAT_BREAKDOWN;
  }
  st.flags |= bad;
  if (!bad) {
    for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
      const int j = e / np, i = e - j * np;
      m.Xd[i + j * ld] = (i <= j && j < n) ? double(m.W[i + j * ld]) : 0.0;
    }
    __syncthreads();
    const auto Xv = xcolmajor<XG>(m.Xd, ld);
    for (;;) {
      // R = A - Xd^T Xd, symmetric: upper tiles computed, mirrored into W
      double sr = 0.0;
      for (int t = wave_id(); t < nt * nt; t += NW) {
        const int I = t / nt, J = t - I * nt;
        if (I > J) continue;
        Tile<double, TB> c;
        tload(c, A64.sub(I * TB, J * TB));
        gemm_sum<Gemm<double, TB, E64>>(c, 0, I + 1, [&](int K) { return Xv.sub(K * TB, I * TB).t(); }, [&](int K) { return Xv.sub(K * TB, J * TB); });
        const double wgt = I == J ? 1.0 : 2.0;
        const int l = lane_id(), j = tcol<TB>(l);
#pragma unroll
        for (int r = 0; r < Tile<double, TB>::EPL; ++r) {
          const int i = trow<double, TB>(l, r);
          const float v = float(c.v[r]);
          m.W[(I * TB + i) + (J * TB + j) * ld] = v;
          m.W[(J * TB + j) + (I * TB + i) * ld] = v;
          sr += wgt * c.v[r] * c.v[r];
        }
      }
      const double eta = sqrt(block_sum<NW>(sr, m.red)) / na;
      if (refine_decide(st, eta, g.tau, g.max_iter)) break;
      // FP32 copy of the factor (padding: identity) for the correction solves
      for (int e = threadIdx.x; e < np * np; e += blockDim.x) {
        const int j = e / np, i = e - j * np;
        m.A1[i + j * ld] = i < n && j < n ? float(m.Xd[i + j * ld]) : (i == j ? 1.0f : 0.0f);
      }
      __syncthreads();
      newton_correction<float, TB, ENG, NW>(xcolmajor<WG>(m.W, ld), xcolmajor<XG>(m.A1, ld), Xv, nt, to_lds(m.wb + wave_id() * wave_scratch(TB)));
      ++st.it;
      __syncthreads();
    }
  }
  __syncthreads();
  int info0 = 0;
  const bool fb = !(st.flags & TLA_STAT_CONVERGED);
  if (!XG && fb) {
    if (threadIdx.x == 0) *m.info = 0;
    ingest<double, NW>(m.Xd, ld, np, Ag, lda, n, +1, 1.0);
    __syncthreads();
    Ctx<double> cd{n, nt, to_lds(reinterpret_cast<double*>(m.wb) + wave_id() * wave_scratch(TB)), to_lds(m.info)};
    constexpr int ENG64 = ENG == ENG_VALU ? ENG_VALU : E64;
    potrf_blocked<double, TB, ENG64, NW, VAR>(xcolmajor<XG>(m.Xd, ld), cd);
    __syncthreads();
    info0 = *m.info;
  }
  if (!(XG && fb)) egress<double, NW, !XG>(Ag, lda, n, m.Xd, ld, 1);
  if (threadIdx.x == 0) *in.info = info0;
  write_stat(in, st);
}

template <int TB, int ENG, int NW, int VAR, bool XG, bool WG = false>
__global__ __launch_bounds__(NW * 64) void k_potrf_mixed(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  potrf_mixed_body<TB, ENG, NW, VAR, XG, WG>(g, fetch_uniform(g, blockIdx.x), smem);
}

}  // namespace tla
