// Solve with the upper Cholesky factor: B := (X^T X)^{-1} B for every
// instance, the consumer of the factorization (Fig. 2a) that the paper's
// motivation lists among the LAPACK building blocks next to it.  One
// workgroup per instance; the factor is read through the caches and B is
// solved in place in global memory.  The right-hand sides are cut into
// 16-column tiles handed to the waves; each wave runs, for its tiles, the
// forward substitution with X^T and then the back substitution with X over
// 16 x 16 tiles: matrix-core products for the updates, the strip tile
// solvers for the diagonal blocks.  A wave reads back only what it wrote.
#include "tla_inplace.hpp"
#include "tla_registry.h"

namespace tla {

// In-place view of an nr x nc column-major matrix: reads outside return 0,
// writes there are dropped.
struct RectView {
  double* p;
  int ld, nr, nc;
  int r0, c0;
  bool tr;
  TLA_DI double operator()(int i, int j) const {
    const int r = tr ? r0 + j : r0 + i, c = tr ? c0 + i : c0 + j;
    const int rr = r < nr ? r : nr - 1, cc = c < nc ? c : nc - 1;
    const double raw = to_gbl(p)[rr + (size_t)cc * ld];
    return (r < nr && c < nc) ? raw : 0.0;
  }
  TLA_DI void store(int i, int j, double v) const {
    const int r = tr ? r0 + j : r0 + i, c = tr ? c0 + i : c0 + j;
    if (r < nr && c < nc) to_gbl(p)[r + (size_t)c * ld] = v;
  }
  TLA_DI void fence() const { __threadfence_block(); }
  TLA_DI RectView sub(int i0, int j0) const {
    RectView v = *this;
    if (tr) { v.r0 += j0; v.c0 += i0; } else { v.r0 += i0; v.c0 += j0; }
    return v;
  }
  TLA_DI RectView t() const { RectView v = *this; v.tr = !tr; return v; }
};

template <int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_potrs(KArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  const int n = g.n[b], m = g.m[b];
  const double* Xg = g.a[b];
  double* Bg = g.c[b];
  const int ldx = g.lda[b], ldb = g.ldc[b];
  int bad = 0;
  if (n < 0 || n > g.n_max || m < 0 || m > g.m_max) bad = -1;
  else if (ldx < (n > 1 ? n : 1) || ldb < (n > 1 ? n : 1)) bad = -2;
  if (bad != 0 || n == 0 || m == 0) {
    if (threadIdx.x == 0) g.info[b] = bad;
    return;
  }
  int* s_info = reinterpret_cast<int*>(smem + NW * wave_scratch(16) * sizeof(double));
  if (threadIdx.x == 0) *s_info = INT_MAX;
  __syncthreads();
  // a zero diagonal entry of the factor: report the first and leave B
  for (int k = threadIdx.x; k < n; k += blockDim.x)
    if (to_gbl(Xg)[k + (size_t)k * ldx] == 0.0) atomicMin(s_info, k + 1);
  __syncthreads();
  const int zero = *s_info;
  if (zero != INT_MAX) {
    if (threadIdx.x == 0) g.info[b] = zero;
    return;
  }
  lds_t<double>* wbuf = to_lds(reinterpret_cast<double*>(smem) + wave_id() * wave_scratch(16));
  const IOView<double> X = ioview<double>(const_cast<double*>(Xg), ldx, n, true);
  const RectView Bv{Bg, ldb, n, m, 0, 0, false};
  const int nt = (n + 15) / 16, mt = (m + 15) / 16;
  typedef Gemm<double, 16, ENG_MFMA> G;
  for (int J = wave_id(); J < mt; J += NW) {
    // Z = X^{-T} B: tile rows top to bottom
    for (int I = 0; I < nt; ++I) {
      Tile<double, 16> c;
      tload(c, Bv.sub(I * 16, J * 16));
      gemm_sum<G>(c, 0, I, [&](int K) { return X.sub(K * 16, I * 16).t(); }, [&](int K) { return Bv.sub(K * 16, J * 16); });
      tile_trsm_ut<double, 16>(c, X.sub(I * 16, I * 16), wbuf);
      tstore(c, Bv.sub(I * 16, J * 16));
    }
    // Y = X^{-1} Z: tile rows bottom to top
    for (int I = nt - 1; I >= 0; --I) {
      Tile<double, 16> c;
      tload(c, Bv.sub(I * 16, J * 16));
      gemm_sum<G>(c, I + 1, nt, [&](int K) { return X.sub(I * 16, K * 16); }, [&](int K) { return Bv.sub(K * 16, J * 16); });
      tile_trsm_u<double>(c, X.sub(I * 16, I * 16), wbuf);
      tstore(c, Bv.sub(I * 16, J * 16));
    }
  }
  if (threadIdx.x == 0) g.info[b] = 0;
}

// Y := I on every valid instance (the right-hand sides of the inverse).
__global__ __launch_bounds__(256) void k_potri_eye(KArgs g) {
  const int b = blockIdx.x;
  const int n = g.n[b], ld = g.ldc[b];
  if (n <= 0 || n > g.n_max || ld < n) return;
  gbl_t<double>* Y = to_gbl(g.c[b]);
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int j = e / n, i = e - j * n;
    Y[i + (size_t)j * ld] = i == j ? 1.0 : 0.0;
  }
}

KFn potri_eye_kernel() { return reinterpret_cast<KFn>(&k_potri_eye); }

KFn potrs_kernel(int nwi) {
  switch (nwi) {
    case 0: return reinterpret_cast<KFn>(&k_potrs<1>);
    case 1: return reinterpret_cast<KFn>(&k_potrs<2>);
    case 2: return reinterpret_cast<KFn>(&k_potrs<4>);
  }
  return nullptr;
}
size_t potrs_lds_bytes(int nw) { return (size_t)nw * wave_scratch(16) * sizeof(double) + 16; }

}  // namespace tla
