// Reduction of general Sylvester and Lyapunov equations to the triangular
// cores (the Bartels-Stewart method).  The paper solves only the triangular
// equations of Fig. 2 and names solvers for Sylvester-like equations as their
// purpose (Motivation paragraph); a user holding general coefficients first
// brings them to triangular form by orthogonal similarity:
//
//   A^T = Z T_A Z^T, B = W T_B W^T (real Schur forms, T_* upper triangular)
//   L = T_A^T (lower), U = T_B (upper)
//   A X + X B = C   <=>  L Y + Y U = Z^T C W,  X = Z Y W^T
//   A X + X A^T = S <=>  L Y + Y L^T = Z^T S Z, X = Z Y Z^T
//
// Three kernels bracket the existing triangular solves:
//   k_schur      one wavefront per matrix: Householder reduction to upper
//                Hessenberg form, then the implicit single-shift QR iteration
//                (Wilkinson shift, deflation on negligible subdiagonal
//                entries, exceptional shifts), the Schur vectors accumulated;
//   k_ge_prep    per instance: status merge and the pointer / size arrays the
//                triangular solves take;
//   k_ge_xform   one workgroup per matrix: the two-sided transforms
//                Z^T M W before and Z M W^T after, as 16 x 16 tile products
//                on the FP64 matrix cores.
// Only real spectra reduce to triangular form with real arithmetic: a
// coefficient whose real Schur form keeps a 2 x 2 block (a complex conjugate
// eigenvalue pair) is reported per instance and left unsolved.
#include <cstdio>
#include <cstdlib>

#include "tla_kernels.hpp"
#include "tla_host.h"

#define GE_HIP(x)                                                                   \
  do {                                                                              \
    hipError_t e_ = (x);                                                            \
    if (e_ != hipSuccess) {                                                         \
      if (getenv("TLA_LOG")) fprintf(stderr, "tla: %s failed: %s\n", #x, hipGetErrorString(e_)); \
      return TLA_E_HIP;                                                             \
    }                                                                               \
  } while (0)

namespace tla {

constexpr int kSchurMaxN = 64;    // one matrix row / column per lane
constexpr int kSchurMaxIts = 60;  // QR iterations without a deflation before the instance is given up

// Per-instance outcomes of the front end (written to info[b]).
constexpr int kGeComplex = -4;    // a coefficient has complex eigenvalues
constexpr int kGeNoConv = -5;     // QR iteration did not converge, or a non-finite coefficient entry

struct SchurSet {
  const double* const* m;  // input matrices, column-major
  const int* ldm;
  int trans;               // factor M^T instead of M
  int lower;               // store T^T (lower triangular) instead of T
  double* t;               // triangular factor: instance b at t + b * stride, leading dimension n_max
  double* q;               // Schur vectors (M or M^T = Q T Q^T), same layout
  int* status;             // int[batch]
};

struct SchurArgs {
  int batch, n_max, nsets;
  const int* n;
  long long stride;
  SchurSet set[2];
};

namespace {

TLA_DI double uni(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readfirstlane((int)b);
  const int hi = __builtin_amdgcn_readfirstlane((int)(b >> 32));
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned)lo);
}

TLA_DI double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return uni(v);
}

// Plane rotation (c, s) with c x + s y = r >= 0 and -s x + c y = 0, scaled
// against overflow; (1, 0) for x = y = 0.
TLA_DI void givens(double x, double y, double& c, double& s) {
  const double m = fmax(fabs(x), fabs(y));
  if (m == 0.0) {
    c = 1.0;
    s = 0.0;
    return;
  }
  const double xs = x / m, ys = y / m;
  const double r = sqrt(xs * xs + ys * ys);
  c = xs / r;
  s = ys / r;
}

// The same rotation without divisions: 1 / sqrt(x^2 + y^2) from the hardware
// estimate refined by two Newton steps; the scaled form above where
// x^2 + y^2 could overflow or lose precision to underflow.
TLA_DI void givens_fast(double x, double y, double& c, double& s) {
  const double r2 = x * x + y * y;
  if (!(r2 > 1e-280 && r2 < 1e280)) {
    givens(x, y, c, s);
    return;
  }
  double ri = __builtin_amdgcn_rsq(r2);
  ri = __builtin_fma(0.5 * ri, __builtin_fma(-r2 * ri, ri, 1.0), ri);
  ri = __builtin_fma(0.5 * ri, __builtin_fma(-r2 * ri, ri, 1.0), ri);
  c = x * ri;
  s = y * ri;
}

// Rotation of rows (k, k+1) over columns j0..n-1 and of columns (k, k+1)
// over rows 0..i1 of H (LDS, leading dimension LD), as the similarity
// H <- G^T H G with G = [[c, -s], [s, c]] in the plane (k, k+1).
template <int LD>
TLA_DI void rotate_h(lds_t<double>* H, int n, int k, int j0, int i1, double c, double s) {
  const int l = lane_id();
  if (l >= j0 && l < n) {
    const double a = H[k + l * LD], b = H[k + 1 + l * LD];
    H[k + l * LD] = c * a + s * b;
    H[k + 1 + l * LD] = c * b - s * a;
  }
  compiler_fence();
  if (l <= i1) {
    const double a = H[l + k * LD], b = H[l + (k + 1) * LD];
    H[l + k * LD] = c * a + s * b;
    H[l + (k + 1) * LD] = c * b - s * a;
  }
  compiler_fence();
}

// Q <- Q G for the rotations recorded in cs (pairs (c, s) at 2k, 2k+1) at
// positions lo..hi-1, in that order; lane i holds row i of Q in q[].  Every
// unused position holds the identity (1, 0), which leaves q exactly as it
// is, so the rotations are applied in chunks of 8 whose (c, s) are loaded
// together, and only chunks that meet [lo, hi) are visited.
template <int NM>
TLA_DI void rotate_q(double (&q)[NM], const lds_t<double>* cs, int lo, int hi) {
  constexpr int CH = 8;
#pragma unroll
  for (int k0 = 0; k0 + 1 < NM; k0 += CH) {
    if (k0 + CH > lo && k0 < hi) {
      double c[CH], s[CH];
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        if (k0 + e + 1 < NM) {
          c[e] = cs[2 * (k0 + e)];
          s[e] = cs[2 * (k0 + e) + 1];
        }
      }
#pragma unroll
      for (int e = 0; e < CH; ++e) {
        const int k = k0 + e;
        if (k + 1 < NM) {
          const double a = q[k], b = q[k + 1];
          q[k] = c[e] * a + s[e] * b;
          q[k + 1] = c[e] * b - s[e] * a;
        }
      }
    }
    compiler_fence();  // one chunk's (c, s) in registers at a time
  }
}

// identity rotations back at positions lo..hi-1
TLA_DI void reset_rotations(lds_t<double>* cs, int lo, int hi) {
  const int l = lane_id();
  if (l >= lo && l < hi) {
    cs[2 * l] = 1.0;
    cs[2 * l + 1] = 0.0;
  }
  compiler_fence();
}

}  // namespace

// NM: largest order handled (16, 32 or 64): the LDS holds H (NM x (NM + 1)),
// each lane holds one row of Q (NM registers).
template <int NM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NM == 64 ? 1 : (NM == 32 ? 2 : 3)))) void
k_schur(SchurArgs g) {
  constexpr int LD = NM + 1;  // odd: row and column walks spread over the banks
  __shared__ double Hs[NM * LD];
  __shared__ double vs_s[64];
  __shared__ double cs_s[2 * NM];
  lds_t<double>* H = to_lds(Hs);
  lds_t<double>* vs = to_lds(vs_s);
  lds_t<double>* cs = to_lds(cs_s);
  const int si = blockIdx.x / g.batch, b = blockIdx.x - si * g.batch;
  const SchurSet S = g.set[si];
  const int l = lane_id();
  const int n = g.n[b];
  if (n < 0 || n > g.n_max) {
    if (l == 0) S.status[b] = -1;
    return;
  }
  const int ldm = S.ldm[b];
  if (ldm < (n > 1 ? n : 1)) {
    if (l == 0) S.status[b] = -2;
    return;
  }
  if (n == 0) {
    if (l == 0) S.status[b] = 0;
    return;
  }
  // ---- ingest: column j of M is read by the lanes (coalesced); M^T is stored transposed
  const gbl_t<double>* M = to_gbl(S.m[b]);
  bool finite = true;
  for (int j = 0; j < n; ++j) {
    if (l < n) {
      const double v = M[l + (size_t)j * ldm];
      finite = finite && __builtin_isfinite(v);
      if (S.trans) H[j + l * LD] = v;
      else H[l + j * LD] = v;
    }
  }
  if (__any(!finite)) {
    if (l == 0) S.status[b] = kGeNoConv;
    return;
  }
  if (l < NM) {
    cs[2 * l] = 1.0;
    cs[2 * l + 1] = 0.0;
  }
  compiler_fence();

  double q[NM];
#pragma unroll
  for (int j = 0; j < NM; ++j) q[j] = l == j ? 1.0 : 0.0;

  // ---- Householder reduction to upper Hessenberg form: H <- P H P, Q <- Q P,
  // P = I - tau v v^T zeroing column k below the subdiagonal (v_{k+1} = 1)
  for (int k = 0; k + 2 < n; ++k) {
    const double xi = (l > k && l < n) ? H[l + k * LD] : 0.0;
    const double ss = wave_sum(l > k + 1 ? xi * xi : 0.0);
    if (ss == 0.0) continue;
    const double alpha = read_lane(xi, k + 1);
    const double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
    const double tau = (beta - alpha) / beta;
    const double sc = 1.0 / (alpha - beta);
    vs[l] = l == k + 1 ? 1.0 : (l > k + 1 ? xi * sc : 0.0);
    compiler_fence();
    // left: rows k+1..n-1 of columns k+1..n-1 (lane = column)
    if (l > k && l < n) {
      double w = 0.0;
      for (int i = k + 1; i < n; ++i) w += vs[i] * H[i + l * LD];
      w *= tau;
      for (int i = k + 1; i < n; ++i) H[i + l * LD] -= vs[i] * w;
      H[l + k * LD] = l == k + 1 ? beta : 0.0;
    }
    compiler_fence();
    // right: columns k+1..n-1 of every row (lane = row)
    if (l < n) {
      double u = 0.0;
      for (int j = k + 1; j < n; ++j) u += H[l + j * LD] * vs[j];
      u *= tau;
      for (int j = k + 1; j < n; ++j) H[l + j * LD] -= u * vs[j];
    }
    double u = 0.0;
#pragma unroll
    for (int j = 0; j < NM; ++j) u += q[j] * vs[j];
    u *= tau;
#pragma unroll
    for (int j = 0; j < NM; ++j) q[j] -= u * vs[j];
    compiler_fence();
  }

  // ---- implicit single-shift QR on the active window [lo, hi]
  const double ulp = 2.220446049250313e-16;           // 2^-52
  const double smlnum = 2.2250738585072014e-308 * ((double)n / ulp);
  int hi = n - 1, its = 0, fail = 0;
  while (hi > 0) {
    // largest l in [1, hi] whose subdiagonal entry is negligible against its
    // diagonal neighbours
    bool neg = false;
    if (l >= 1 && l <= hi) {
      const double sub = fabs(H[l + (l - 1) * LD]);
      double tst = fabs(H[(l - 1) + (l - 1) * LD]) + fabs(H[l + l * LD]);
      if (tst == 0.0) {
        if (l >= 2) tst += fabs(H[(l - 1) + (l - 2) * LD]);
        if (l + 1 <= hi) tst += fabs(H[(l + 1) + l * LD]);
      }
      neg = sub <= smlnum || sub <= ulp * tst;
    }
    const unsigned long long mask = __ballot(neg);
    const int lo = mask ? 63 - __clzll(mask) : 0;
    compiler_fence();
    if (lo > 0 && l == 0) H[lo + (lo - 1) * LD] = 0.0;
    compiler_fence();
    if (lo == hi) {  // 1 x 1 block: an eigenvalue
      hi -= 1;
      its = 0;
      continue;
    }
    if (lo == hi - 1) {  // 2 x 2 block: split it if its eigenvalues are real
      const double a = uni(H[lo + lo * LD]), bq = uni(H[lo + hi * LD]);
      const double e = uni(H[hi + lo * LD]), d = uni(H[hi + hi * LD]);
      const double p = 0.5 * (a - d), disc = p * p + bq * e;
      if (disc < 0.0) {
        fail = kGeComplex;
        break;
      }
      if (e != 0.0) {
        // (z, e) is an eigenvector for the eigenvalue d + z: the rotation whose
        // first column it spans makes the block upper triangular
        const double z = p + copysign(sqrt(disc), p);
        double c, s;
        givens(z, e, c, s);
        compiler_fence();
        rotate_h<LD>(H, n, lo, lo, hi, c, s);
        if (l == 0) {
          cs[2 * lo] = c;
          cs[2 * lo + 1] = s;
          H[hi + lo * LD] = 0.0;
        }
        compiler_fence();
        rotate_q<NM>(q, cs, lo, lo + 1);
        compiler_fence();
        reset_rotations(cs, lo, lo + 1);
      }
      hi -= 2;
      its = 0;
      continue;
    }
    if (++its > kSchurMaxIts) {
      // no deflation: a complex pair at the bottom of the window, or no convergence
      const double a = uni(H[(hi - 1) + (hi - 1) * LD]), bq = uni(H[(hi - 1) + hi * LD]);
      const double e = uni(H[hi + (hi - 1) * LD]), d = uni(H[hi + hi * LD]);
      const double p = 0.5 * (a - d);
      fail = p * p + bq * e < 0.0 ? kGeComplex : kGeNoConv;
      break;
    }
    // shift: the eigenvalue of the trailing 2 x 2 block nearer its last
    // diagonal entry (Wilkinson), its last diagonal entry when that block has
    // complex eigenvalues, and an ad hoc exceptional shift every 10th step
    const double a = uni(H[(hi - 1) + (hi - 1) * LD]), bq = uni(H[(hi - 1) + hi * LD]);
    const double e = uni(H[hi + (hi - 1) * LD]), d = uni(H[hi + hi * LD]);
    double sigma;
    if (its % 10 == 0) {
      sigma = d + 0.75 * fabs(e);
    } else {
      const double p = 0.5 * (a - d), disc = p * p + bq * e;
      sigma = d;
      if (disc >= 0.0) {
        const double z = p + copysign(sqrt(disc), p);
        if (z != 0.0) sigma = d - bq * e / z;
      }
    }
    // the sweep: the first rotation from the shifted first column, then the
    // bulge chased down the window.  Rotation k updates rows (k, k+1) (lane =
    // column) and then columns (k, k+1) (lane = row).  Both operand pairs are
    // read before either update: the row update changes no column operand
    // except those of rows k and k+1, which lanes k and k+1 take from the row
    // update's results (cross-lane reads), and the next rotation's pair
    // (h_{k+1,k}, h_{k+2,k}) comes from the column update's results the same
    // way; the LDS then carries only the stores, and the loads of the next
    // rotation overlap the computation of its (c, s).
    double x = uni(H[lo + lo * LD]) - sigma, y = uni(H[(lo + 1) + lo * LD]);
    compiler_fence();
    for (int k = lo; k < hi; ++k) {
      const int j0 = k > lo ? k - 1 : lo;
      const int i1 = k + 2 < hi ? k + 2 : hi;
      const bool rl = l >= j0 && l < n, cl = l <= i1;
      const int lr = l < n ? l : n - 1;
      const double ra = H[k + lr * LD], rb = H[(k + 1) + lr * LD];
      double ca = H[lr + k * LD], cb = H[lr + (k + 1) * LD];
      double c, s;
      givens_fast(x, y, c, s);
      const double ra2 = c * ra + s * rb;
      double rb2 = c * rb - s * ra;
      if (k > lo && l == k - 1) rb2 = 0.0;  // the annihilated bulge
      if (rl) {
        H[k + l * LD] = ra2;
        H[(k + 1) + l * LD] = rb2;
      }
      const double h00 = read_lane(ra2, k), h01 = read_lane(ra2, k + 1);
      const double h10 = read_lane(rb2, k), h11 = read_lane(rb2, k + 1);
      if (l == k) {
        ca = h00;
        cb = h01;
      } else if (l == k + 1) {
        ca = h10;
        cb = h11;
      }
      const double ca2 = c * ca + s * cb, cb2 = c * cb - s * ca;
      if (cl) {
        H[l + k * LD] = ca2;
        H[l + (k + 1) * LD] = cb2;
      }
      if (l == 0) {
        cs[2 * k] = c;
        cs[2 * k + 1] = s;
      }
      if (k + 1 < hi) {
        x = read_lane(ca2, k + 1);
        y = read_lane(ca2, k + 2);
      }
      compiler_fence();
    }
    rotate_q<NM>(q, cs, lo, hi);
    compiler_fence();
    reset_rotations(cs, lo, hi);
  }
  if (fail != 0) {
    if (l == 0) S.status[b] = fail;
    return;
  }
  // ---- egress: T (or T^T) with exact zeros off its triangle, and Q
  gbl_t<double>* T = to_gbl(S.t + (size_t)b * g.stride);
  gbl_t<double>* Q = to_gbl(S.q + (size_t)b * g.stride);
  const int ld = g.n_max;
  for (int j = 0; j < n; ++j) {
    if (l < n) {
      double v;
      if (S.lower) v = l >= j ? H[j + l * LD] : 0.0;
      else v = l <= j ? H[l + j * LD] : 0.0;
      T[l + (size_t)j * ld] = v;
    }
  }
#pragma unroll
  for (int j = 0; j < NM; ++j)
    if (j < n && l < n) Q[l + (size_t)j * ld] = q[j];
  if (l == 0) S.status[b] = 0;
}

// ------------------------------------------------------------ prep
struct GePrepArgs {
  int batch, n_max, nsets;
  const int* n;
  const int* st0;       // status of the first coefficient
  const int* st1;       // status of the second (Sylvester) or null
  const int* ldc;
  int* gstat;           // merged status
  int* n_eff;           // n[b] where the front end succeeded, else 0
  int* ldw;             // n_max: leading dimension of the workspace matrices
  const double** lp;    // L_b
  const double** up;    // U_b (Sylvester)
  double* lbase;
  double* ubase;
  long long stride;
};

__global__ void k_ge_prep(GePrepArgs g) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= g.batch) return;
  int st = g.st0[b];
  if (st == 0 && g.st1) st = g.st1[b];
  const int n = g.n[b];
  if (st == 0 && g.ldc[b] < (n > 1 ? n : 1)) st = -2;
  g.gstat[b] = st;
  g.n_eff[b] = st == 0 ? n : 0;
  g.ldw[b] = g.n_max > 0 ? g.n_max : 1;
  g.lp[b] = g.lbase + (size_t)b * g.stride;
  if (g.up) g.up[b] = g.ubase + (size_t)b * g.stride;
}

// ------------------------------------------------------------ transforms
// Element (i, j) of an n x n column-major matrix at p, or of its transpose;
// with sym, of the symmetric matrix given by its lower triangle.  Zero
// outside n x n.
template <bool LDS>
struct MView {
  using P = std::conditional_t<LDS, const lds_t<double>*, const gbl_t<double>*>;
  P p;
  int ld, n, r0, c0;
  bool tr, sym;
  TLA_DI double operator()(int i, int j) const {
    int r = r0 + i, c = c0 + j;
    if (tr) {
      const int t = r;
      r = c;
      c = t;
    }
    const bool in = r < n && c < n;
    if (sym && r < c) {
      const int t = r;
      r = c;
      c = t;
    }
    const int rr = r < n ? r : n - 1, cc = c < n ? c : n - 1;
    const double v = p[rr + (size_t)cc * ld];
    return in ? v : 0.0;
  }
  TLA_DI MView sub(int i0, int j0) const {
    MView v = *this;
    v.r0 += i0;
    v.c0 += j0;
    return v;
  }
};

struct XformArgs {
  int batch, n_max;
  const int* n;
  const int* gstat;
  double* const* c;     // the caller's right-hand sides, overwritten
  const int* ldc;
  const double* p;      // left factor Z
  const double* r;      // right factor W (Sylvester) or Z (Lyapunov)
  long long stride;
  int fwd;              // 1: Z^T M W, 0: Z M W^T
  int sym;              // Lyapunov: M symmetric (lower triangle read when fwd), result symmetrised
  int* info;            // backward pass: the front end's status where nonzero
};

template <int NW>
__global__ __launch_bounds__(NW * 64) void k_ge_xform(XformArgs g) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int b = blockIdx.x;
  const int st = g.gstat[b];
  if (st != 0) {
    if (!g.fwd && threadIdx.x == 0) g.info[b] = st;
    return;
  }
  const int n = g.n[b];
  if (n == 0) return;
  const int ld = g.ldc[b];
  const int nt = (n + 15) / 16, ldt = 16 * nt + 1;
  lds_t<double>* T = to_lds(reinterpret_cast<double*>(smem));
  double* Cg = g.c[b];
  const double* P = g.p + (size_t)b * g.stride;
  const double* R = g.r + (size_t)b * g.stride;
  const int w = wave_id(), l = lane_id();
  // phase 1: T = op(P) M, op(P) = P^T forward, P backward
  MView<false> Pv{to_gbl(P), g.n_max, n, 0, 0, g.fwd != 0, false};
  MView<false> Mv{to_gbl(static_cast<const double*>(Cg)), ld, n, 0, 0, false, g.sym != 0 && g.fwd != 0};
  for (int t = w; t < nt * nt; t += NW) {
    const int ti = t % nt, tj = t / nt;
    Tile<double, 16> acc;
    tzero(acc);
    for (int k = 0; k < nt; ++k) Gemm<double, 16, ENG_MFMA>::sub(acc, Pv.sub(16 * ti, 16 * k), Mv.sub(16 * k, 16 * tj));
#pragma unroll
    for (int r = 0; r < 4; ++r) T[16 * ti + trow<double, 16>(l, r) + (16 * tj + tcol<16>(l)) * ldt] = -acc.v[r];
  }
  __syncthreads();
  // phase 2: out = T op(R), op(R) = R forward, R^T backward; written over C
  MView<true> Tv{T, ldt, 16 * nt, 0, 0, false, false};
  MView<false> Rv{to_gbl(R), g.n_max, n, 0, 0, g.fwd == 0, false};
  gbl_t<double>* Co = to_gbl(Cg);
  for (int t = w; t < nt * nt; t += NW) {
    const int ti = t % nt, tj = t / nt;
    if (g.sym && ti < tj) continue;  // symmetric result: lower tiles, mirrored on store
    Tile<double, 16> acc;
    tzero(acc);
    for (int k = 0; k < nt; ++k) Gemm<double, 16, ENG_MFMA>::sub(acc, Tv.sub(16 * ti, 16 * k), Rv.sub(16 * k, 16 * tj));
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int i = 16 * ti + trow<double, 16>(l, r), j = 16 * tj + tcol<16>(l);
      if (i < n && j < n) {
        if (!g.sym) {
          Co[i + (size_t)j * ld] = -acc.v[r];
        } else if (i >= j) {
          Co[i + (size_t)j * ld] = -acc.v[r];
          Co[j + (size_t)i * ld] = -acc.v[r];
        }
      }
    }
  }
}

// ------------------------------------------------------------ host side
namespace {

constexpr int kXformNW = 4;

// Front-end workspace: `mats` n_max x n_max FP64 matrices per instance, then
// the pointer and integer arrays.
struct GeLayout {
  size_t mat_off, ptr_off, int_off, bytes;
  long long stride;
};

GeLayout ge_layout(int batch, int n_max, int mats) {
  GeLayout L{};
  L.stride = (long long)n_max * n_max;
  L.mat_off = 0;
  const size_t mat_bytes = (size_t)batch * mats * L.stride * sizeof(double);
  L.ptr_off = (mat_bytes + 255) & ~(size_t)255;
  const size_t ptr_bytes = (size_t)2 * batch * sizeof(double*);
  L.int_off = (L.ptr_off + ptr_bytes + 255) & ~(size_t)255;
  L.bytes = L.int_off + (size_t)6 * batch * sizeof(int);
  return L;
}

tla_status ensure_ge(tla_ctx* h, size_t bytes) {
  if (bytes <= h->ge_bytes) return TLA_OK;
  if (h->ge_work) {
    GE_HIP(hipStreamSynchronize(h->stream));
    hipFree(h->ge_work);
    h->ge_work = nullptr;
    h->ge_bytes = 0;
  }
  if (hipMalloc(&h->ge_work, bytes) != hipSuccess) return TLA_E_NOMEM;
  h->ge_bytes = bytes;
  return TLA_OK;
}

tla_status ge_checks(tla_handle h, tla_prec prec, int batch, int n_max) {
  if (!h || batch < 0 || n_max < 0) return TLA_E_ARG;
  if (prec < TLA_F64 || prec > TLA_MIXED_BF16) return TLA_E_ARG;
  if (n_max > kSchurMaxN) return TLA_E_UNSUPPORTED;
  return TLA_OK;
}

// One front-end call: op TLA_TRSYL (A, B, C) or TLA_TRLYAP (A, S).
tla_status ge_solve(tla_ctx* h, int op, tla_prec prec, int batch, int n_max, const int* n,
                    const double* const* A, const int* lda, const double* const* B, const int* ldb,
                    double* const* C, const int* ldc, int* info, tla_stat* stat) {
  GE_HIP(hipSetDevice(h->device));
  const bool syl = op == TLA_TRSYL;
  const int mats = syl ? 4 : 2;
  const int nm = n_max > 0 ? n_max : 1;
  const GeLayout Lo = ge_layout(batch, nm, mats);
  tla_status s = ensure_ge(h, Lo.bytes);
  if (s != TLA_OK) return s;
  char* base = reinterpret_cast<char*>(h->ge_work);
  double* mat = reinterpret_cast<double*>(base + Lo.mat_off);
  double* Zq = mat;                                   // Schur vectors of A^T
  double* Lt = mat + (size_t)batch * Lo.stride;       // L = T_A^T
  double* Wq = syl ? mat + (size_t)2 * batch * Lo.stride : Zq;
  double* Ut = syl ? mat + (size_t)3 * batch * Lo.stride : nullptr;
  const double** lp = reinterpret_cast<const double**>(base + Lo.ptr_off);
  const double** up = lp + batch;
  int* ints = reinterpret_cast<int*>(base + Lo.int_off);
  int* st0 = ints;
  int* st1 = ints + batch;
  int* gstat = ints + 2 * batch;
  int* n_eff = ints + 3 * batch;
  int* ldw = ints + 4 * batch;

  SchurArgs sa{};
  sa.batch = batch;
  sa.n_max = nm;
  sa.nsets = syl ? 2 : 1;
  sa.n = n;
  sa.stride = Lo.stride;
  sa.set[0] = SchurSet{A, lda, 1, 1, Lt, Zq, st0};
  if (syl) sa.set[1] = SchurSet{B, ldb, 0, 0, Ut, Wq, st1};
  const dim3 sg(batch * sa.nsets);
  if (nm <= 16) hipLaunchKernelGGL(k_schur<16>, sg, dim3(64), 0, h->stream, sa);
  else if (nm <= 32) hipLaunchKernelGGL(k_schur<32>, sg, dim3(64), 0, h->stream, sa);
  else hipLaunchKernelGGL(k_schur<64>, sg, dim3(64), 0, h->stream, sa);
  GE_HIP(hipGetLastError());

  GePrepArgs pa{};
  pa.batch = batch;
  pa.n_max = nm;
  pa.n = n;
  pa.st0 = st0;
  pa.st1 = syl ? st1 : nullptr;
  pa.ldc = ldc;
  pa.gstat = gstat;
  pa.n_eff = n_eff;
  pa.ldw = ldw;
  pa.lp = lp;
  pa.up = syl ? up : nullptr;
  pa.lbase = Lt;
  pa.ubase = Ut;
  pa.stride = Lo.stride;
  hipLaunchKernelGGL(k_ge_prep, dim3((batch + 255) / 256), dim3(256), 0, h->stream, pa);
  GE_HIP(hipGetLastError());

  XformArgs xa{};
  xa.batch = batch;
  xa.n_max = nm;
  xa.n = n;
  xa.gstat = gstat;
  xa.c = C;
  xa.ldc = ldc;
  xa.p = Zq;
  xa.r = Wq;
  xa.stride = Lo.stride;
  xa.fwd = 1;
  xa.sym = syl ? 0 : 1;
  xa.info = info;
  const int ntm = (nm + 15) / 16;
  const size_t lds = (size_t)16 * ntm * (16 * ntm + 1) * sizeof(double);
  hipLaunchKernelGGL(k_ge_xform<kXformNW>, dim3(batch), dim3(64 * kXformNW), lds, h->stream, xa);
  GE_HIP(hipGetLastError());

  // the triangular core on the transformed right-hand sides, in place
  if (syl) s = tla_trsyl_batched(h, prec, batch, n_max, n_eff, lp, ldw, up, ldw, C, ldc, info, stat);
  else s = tla_trlyap_batched(h, prec, batch, n_max, n_eff, lp, ldw, C, ldc, info, stat);
  if (s != TLA_OK) return s;

  xa.fwd = 0;
  hipLaunchKernelGGL(k_ge_xform<kXformNW>, dim3(batch), dim3(64 * kXformNW), lds, h->stream, xa);
  GE_HIP(hipGetLastError());
  return TLA_OK;
}

}  // namespace

}  // namespace tla

using namespace tla;

extern "C" tla_status tla_gesyl_batched(tla_handle h, tla_prec prec, int batch, int n_max, const int* n,
                                        const double* const* A, const int* lda, const double* const* B,
                                        const int* ldb, double* const* C, const int* ldc, int* info,
                                        tla_stat* stat) {
  tla_status s = ge_checks(h, prec, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (!n || !A || !lda || !B || !ldb || !C || !ldc || !info) return TLA_E_ARG;
  return ge_solve(h, TLA_TRSYL, prec, batch, n_max, n, A, lda, B, ldb, C, ldc, info, stat);
}

extern "C" tla_status tla_gelyap_batched(tla_handle h, tla_prec prec, int batch, int n_max, const int* n,
                                         const double* const* A, const int* lda, double* const* S,
                                         const int* lds, int* info, tla_stat* stat) {
  tla_status s = ge_checks(h, prec, batch, n_max);
  if (s != TLA_OK || batch == 0) return s;
  if (!n || !A || !lda || !S || !lds || !info) return TLA_E_ARG;
  return ge_solve(h, TLA_TRLYAP, prec, batch, n_max, n, A, lda, nullptr, nullptr, S, lds, info, stat);
}
