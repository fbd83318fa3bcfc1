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
// Four kernels bracket the existing triangular solves:
//   k_hess       one wavefront per matrix: Householder reduction to upper
//                Hessenberg form (dense matrix in LDS), the Schur vectors
//                started;
//   k_schur_qr   one wavefront per matrix: the implicit single-shift QR
//                iteration (Wilkinson shift, deflation on negligible
//                subdiagonal entries, exceptional shifts) on the Hessenberg
//                matrix packed in LDS, the Schur vectors accumulated;
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
  int* esc;                // int[batch]: T was formed scaled by 2^-esc[b]
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

// c a + s b and c b - s a, each rounded the same way wherever it is formed:
// the bulge chase keeps a copy of the entries it needs next in every lane and
// must reproduce the stored values bit for bit.
TLA_DI double rot_hi(double c, double s, double a, double b) { return __builtin_fma(c, a, s * b); }
TLA_DI double rot_lo(double c, double s, double a, double b) { return __builtin_fma(c, b, -(s * a)); }

// The rotation of the bulge chase without divisions or branches: 1 / sqrt(x^2
// + y^2) from the hardware estimate refined by two Newton steps, the second
// folded into the products x / r and y / r.  The matrix is scaled at ingest so
// that its largest entry lies in [1/2, 1): x^2 + y^2 cannot overflow.  x is
// first moved by 2^-500 away from zero, which leaves every |x| >= 2^-446
// unchanged (less than half its last place) and keeps x^2 + y^2 >= 2^-1000:
// a pair below that (far under the working precision of such a matrix) gets a
// rotation onto (x', y): c = +-1, s = 0 for x = +-0, y = 0.
TLA_DI void givens_chase(double x, double y, double& c, double& s) {
  const double xe = x + copysign(0x1p-500, x);
  const double r2 = __builtin_fma(xe, xe, y * y);
  const double r2h = 0.5 * r2;  // the halves of the Newton steps, exact
  double ri = __builtin_amdgcn_rsq(r2);
  ri = __builtin_fma(ri, __builtin_fma(-r2h * ri, ri, 0.5), ri);
  const double h = __builtin_fma(-r2h * ri, ri, 0.5);
  const double cx = xe * ri, sy = y * ri;
  c = __builtin_fma(cx, h, cx);
  s = __builtin_fma(sy, h, sy);
}

TLA_DI double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return uni(v);
}

// Column j of the Hessenberg matrix during the bulge chase has its nonzeros
// in rows 0..j+1 and the bulge in row j+2: stored packed by columns, rows
// 0..j+2 of column j at pk(0, j) + i.
TLA_DI int pk(int i, int j) { return ((j * (j + 5)) >> 1) + i; }

// Rotation of rows (k, k+1) over columns k..n-1 and of columns (k, k+1) over
// rows 0..k+1 of the packed H, as the similarity H <- G^T H G with
// G = [[c, -s], [s, c]] in the plane (k, k+1) (the split of a 2 x 2 block).
TLA_DI void rotate_pk(lds_t<double>* H, int n, int k, double c, double s) {
  const int l = lane_id();
  if (l >= k && l < n) {
    const double a = H[pk(k, l)], b = H[pk(k + 1, l)];
    H[pk(k, l)] = c * a + s * b;
    H[pk(k + 1, l)] = c * b - s * a;
  }
  compiler_fence();
  if (l <= k + 1) {
    const double a = H[pk(l, k)], b = H[pk(l, k + 1)];
    H[pk(l, k)] = c * a + s * b;
    H[pk(l, k + 1)] = c * b - s * a;
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

// ------------------------------------------------------------ Hessenberg
// NM: largest order handled (16, 32 or 64); NW: waves per matrix (1 or 2).
// The LDS holds the dense matrix (NM x (NM + 1)).  With two waves each wave
// takes every other row (left update) and column (right update) of a
// reflector and every other column of Q, and the two partial dot products are
// added through LDS: the serial chains of a step are half as long and twice as
// many waves share a SIMD (the LDS allows four matrices per compute unit at
// NM = 64).  Each lane holds its row of the wave's Q columns in registers.
// Output: H = Q^T M Q (upper Hessenberg, exact zeros below the subdiagonal,
// scaled by 2^-esc) in the T slot, Q in the Q slot, esc, and the status (0, or
// the argument / non-finite code that ends the instance).
template <int NW>
TLA_DI void group_sync() {
  if constexpr (NW > 1) __syncthreads();
  else compiler_fence();
}

template <int NM, int NW>
__global__ __launch_bounds__(64 * NW) __attribute__((amdgpu_waves_per_eu(NW == 2 ? 2 : (NM == 64 ? 1 : (NM == 32 ? 4 : 5))))) void
k_hess(SchurArgs g) {
  constexpr int LD = NM + 1;  // odd: row and column walks spread over the banks
  constexpr int QN = NM / NW; // Schur-vector columns per wave: j = NW m + w
  __shared__ double Hs[NM * LD];
  __shared__ double vs_s[64];
  __shared__ double px_s[2 * 64 * NW];  // the waves' partial dot products (matrix, Q)
  __shared__ double red_s[2 * NW];
  lds_t<double>* H = to_lds(Hs);
  lds_t<double>* vs = to_lds(vs_s);
  lds_t<double>* px = to_lds(px_s);
  lds_t<double>* pq = px + 64 * NW;
  const int si = blockIdx.x / g.batch, b = blockIdx.x - si * g.batch;
  const SchurSet S = g.set[si];
  const int l = lane_id(), w = NW > 1 ? (int)(threadIdx.x >> 6) : 0;
  const bool t0 = threadIdx.x == 0;
  const int n = g.n[b];
  if (n < 0 || n > g.n_max) {
    if (t0) S.status[b] = -1;
    return;
  }
  const int ldm = S.ldm[b];
  if (ldm < (n > 1 ? n : 1)) {
    if (t0) S.status[b] = -2;
    return;
  }
  if (n == 0) {
    if (t0) S.status[b] = 0;
    return;
  }
  // ---- ingest: column j of M is read by the lanes (coalesced), the waves
  // taking every other column; M^T is stored transposed
  const gbl_t<double>* M = to_gbl(S.m[b]);
  bool finite = true;
  double amax = 0.0;
  for (int j = w; j < n; j += NW) {
    if (l < n) {
      const double v = M[l + (size_t)j * ldm];
      finite = finite && __builtin_isfinite(v);
      amax = fmax(amax, fabs(v));
      if (S.trans) H[j + l * LD] = v;
      else H[l + j * LD] = v;
    }
  }
  amax = wave_max(amax);
  const bool bad = __any(!finite);
  if constexpr (NW > 1) {
    if (l == 0) {
      red_s[w] = amax;
      red_s[NW + w] = bad ? 1.0 : 0.0;
    }
    __syncthreads();
    amax = fmax(red_s[0], red_s[1]);
    if (red_s[NW] + red_s[NW + 1] != 0.0) {
      if (t0) S.status[b] = kGeNoConv;
      return;
    }
  } else if (bad) {
    if (t0) S.status[b] = kGeNoConv;
    return;
  }
  // scale by a power of two (exact) so that the largest entry lies in [1/2, 1);
  // T is scaled back at the end, the Schur vectors do not depend on it
  int esc = 0;
  if (amax > 0.0) frexp(amax, &esc);
  group_sync<NW>();
  if (esc != 0 && l < n)
    for (int j = w; j < n; j += NW) H[l + j * LD] = ldexp(H[l + j * LD], -esc);
  group_sync<NW>();

  double q[QN];
#pragma unroll
  for (int m = 0; m < QN; ++m) q[m] = l == NW * m + w ? 1.0 : 0.0;

  // ---- Householder reduction to upper Hessenberg form: H <- P H P, Q <- Q P,
  // P = I - tau v v^T zeroing column k below the subdiagonal (v_{k+1} = 1)
  for (int k = 0; k + 2 < n; ++k) {
    const double xi = (l > k && l < n) ? H[l + k * LD] : 0.0;
    const double ss = wave_sum(l > k + 1 ? xi * xi : 0.0);
    if (ss == 0.0) continue;  // the same in both waves
    const double alpha = read_lane(xi, k + 1);
    const double beta = -copysign(sqrt(alpha * alpha + ss), alpha);
    const double tau = (beta - alpha) / beta;
    const double sc = 1.0 / (alpha - beta);
    if (w == 0) vs[l] = l == k + 1 ? 1.0 : (l > k + 1 ? xi * sc : 0.0);
    group_sync<NW>();
    // left: rows k+1..n-1 of columns k+1..n-1 (lane = column, the wave's rows);
    // the dot products run as four interleaved partial sums
    auto left_dot = [&]() {
      double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
      int i = k + 1 + w;
#pragma unroll 2
      for (; i + 3 * NW < n; i += 4 * NW) {
        w0 += vs[i] * H[i + l * LD];
        w1 += vs[i + NW] * H[i + NW + l * LD];
        w2 += vs[i + 2 * NW] * H[i + 2 * NW + l * LD];
        w3 += vs[i + 3 * NW] * H[i + 3 * NW + l * LD];
      }
      for (; i < n; i += NW) w0 += vs[i] * H[i + l * LD];
      return (w0 + w1) + (w2 + w3);
    };
    auto left_update = [&](double wl) {
#pragma unroll 8
      for (int i = k + 1 + w; i < n; i += NW) H[i + l * LD] -= vs[i] * wl;
      if (w == 0) H[l + k * LD] = l == k + 1 ? beta : 0.0;
    };
    // right: columns k+1..n-1 of every row (lane = row, the wave's columns),
    // and the Schur vectors' dot products (the wave's columns of Q)
    auto right_dot = [&]() {
      double u0 = 0.0, u1 = 0.0, u2 = 0.0, u3 = 0.0;
      int j = k + 1 + w;
#pragma unroll 2
      for (; j + 3 * NW < n; j += 4 * NW) {
        u0 += H[l + j * LD] * vs[j];
        u1 += H[l + (j + NW) * LD] * vs[j + NW];
        u2 += H[l + (j + 2 * NW) * LD] * vs[j + 2 * NW];
        u3 += H[l + (j + 3 * NW) * LD] * vs[j + 3 * NW];
      }
      for (; j < n; j += NW) u0 += H[l + j * LD] * vs[j];
      return (u0 + u1) + (u2 + u3);
    };
    auto right_update = [&](double u) {
#pragma unroll 8
      for (int j = k + 1 + w; j < n; j += NW) H[l + j * LD] -= u * vs[j];
    };
    auto qdot = [&]() {
      double uq[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int m = 0; m < QN; ++m) {
        uq[m & 3] += q[m] * vs[NW * m + w];
        if ((m & 15) == 15) compiler_fence();  // a bounded number of v loads in flight
      }
      return (uq[0] + uq[1]) + (uq[2] + uq[3]);
    };
    double uqt;
    if constexpr (NW == 1) {
      if (l > k && l < n) left_update(tau * left_dot());
      compiler_fence();
      if (l < n) right_update(tau * right_dot());
      uqt = qdot();
    } else {
      // the waves' partial sums are added through LDS (in a fixed order)
      px[64 * w + l] = (l > k && l < n) ? left_dot() : 0.0;
      __syncthreads();
      if (l > k && l < n) left_update(tau * (px[l] + px[64 + l]));
      __syncthreads();
      px[64 * w + l] = l < n ? right_dot() : 0.0;
      pq[64 * w + l] = qdot();
      __syncthreads();
      if (l < n) right_update(tau * (px[l] + px[64 + l]));
      uqt = pq[l] + pq[64 + l];
    }
    uqt *= tau;
#pragma unroll
    for (int m = 0; m < QN; ++m) {
      q[m] -= uqt * vs[NW * m + w];
      if ((m & 15) == 15) compiler_fence();
    }
    group_sync<NW>();
  }
  // ---- hand-off to the QR kernel through the output slots
  gbl_t<double>* T = to_gbl(S.t + (size_t)b * g.stride);
  gbl_t<double>* Q = to_gbl(S.q + (size_t)b * g.stride);
  const int ld = g.n_max;
  for (int j = w; j < n; j += NW)
    if (l < n) T[l + (size_t)j * ld] = H[l + j * LD];
#pragma unroll
  for (int m = 0; m < QN; ++m) {
    const int j = NW * m + w;
    if (j < n && l < n) Q[l + (size_t)j * ld] = q[m];
  }
  if (t0) {
    S.esc[b] = esc;
    S.status[b] = 0;
  }
}

// ------------------------------------------------------------ QR iteration
// NM: largest order handled (16, 32 or 64).  One wave per matrix, the packed
// Hessenberg matrix in LDS (NM (NM + 5) / 2 doubles: two waves per SIMD at
// NM = 64), each lane one row of Q in registers.  Takes the Hessenberg kernel's
// output from the T and Q slots and leaves T (or T^T) and Q there.
template <int NM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(NM == 64 ? 2 : (NM == 32 ? 3 : 4)))) void
k_schur_qr(SchurArgs g) {
  constexpr int PS = NM * (NM + 5) / 2;
  __shared__ double Hs[PS];
  __shared__ double cs_s[2 * NM];
  __shared__ double junk_s[2 * 64 + 2];  // target of the stores of lanes outside a rotation's range
  lds_t<double>* H = to_lds(Hs);
  lds_t<double>* cs = to_lds(cs_s);
  lds_t<double>* J = to_lds(junk_s);
  const int si = blockIdx.x / g.batch, b = blockIdx.x - si * g.batch;
  const SchurSet S = g.set[si];
  const int l = lane_id();
  const int n = g.n[b];
  if (n < 1 || n > g.n_max || S.status[b] != 0) return;  // ended by the Hessenberg kernel (or empty)
  gbl_t<double>* T = to_gbl(S.t + (size_t)b * g.stride);
  gbl_t<double>* Q = to_gbl(S.q + (size_t)b * g.stride);
  const int ld = g.n_max;
  const int esc = S.esc[b];
  // ---- ingest: the Hessenberg part of column j (lane = row), a zero bulge slot below it
  for (int j = 0; j < n; ++j) {
    if (l <= j + 1 && l < n) H[pk(l, j)] = T[l + (size_t)j * ld];
    else if (l <= j + 2) H[pk(l, j)] = 0.0;
  }
  // rows and columns past n are read clamped (in the slot, never used nor stored)
  double q[NM];
  {
    const gbl_t<double>* Qp = Q + (l < n ? l : n - 1);
#pragma unroll
    for (int j = 0; j < NM; ++j) {
      q[j] = *Qp;
      if (j + 1 < n) Qp += ld;
      if ((j & 7) == 7) compiler_fence();  // eight loads in flight at a time
    }
  }
  if (l < NM) {
    cs[2 * l] = 1.0;
    cs[2 * l + 1] = 0.0;
  }
  compiler_fence();

  // ---- implicit single-shift QR on the active window [lo, hi]
  const double ulp = 2.220446049250313e-16;           // 2^-52
  const double smlnum = 2.2250738585072014e-308 * ((double)n / ulp);
  int hi = n - 1, its = 0, fail = 0;
  while (hi > 0) {
    // largest l in [1, hi] whose subdiagonal entry is negligible against its
    // diagonal neighbours
    bool neg = false;
    if (l >= 1 && l <= hi) {
      const double sub = fabs(H[pk(l, l - 1)]);
      double tst = fabs(H[pk(l - 1, l - 1)]) + fabs(H[pk(l, l)]);
      if (tst == 0.0) {
        if (l >= 2) tst += fabs(H[pk(l - 1, l - 2)]);
        if (l + 1 <= hi) tst += fabs(H[pk(l + 1, l)]);
      }
      neg = sub <= smlnum || sub <= ulp * tst;
    }
    const unsigned long long mask = __ballot(neg);
    const int lo = mask ? 63 - __clzll(mask) : 0;
    compiler_fence();
    if (lo > 0 && l == 0) H[pk(lo, lo - 1)] = 0.0;
    compiler_fence();
    int rlo = 0, rhi = 0;  // rotations of this step, recorded in cs at rlo..rhi-1
    if (lo == hi) {  // 1 x 1 block: an eigenvalue
      hi -= 1;
      its = 0;
    } else if (lo == hi - 1) {  // 2 x 2 block: split it if its eigenvalues are real
      const double a = uni(H[pk(lo, lo)]), bq = uni(H[pk(lo, hi)]);
      const double e = uni(H[pk(hi, lo)]), d = uni(H[pk(hi, hi)]);
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
        rotate_pk(H, n, lo, c, s);
        if (l == 0) {
          cs[2 * lo] = c;
          cs[2 * lo + 1] = s;
          H[pk(hi, lo)] = 0.0;
        }
        rlo = lo;
        rhi = lo + 1;
      }
      hi -= 2;
      its = 0;
    } else {
      if (++its > kSchurMaxIts) {
        // no deflation: a complex pair at the bottom of the window, or no convergence
        const double a = uni(H[pk(hi - 1, hi - 1)]), bq = uni(H[pk(hi - 1, hi)]);
        const double e = uni(H[pk(hi, hi - 1)]), d = uni(H[pk(hi, hi)]);
        const double p = 0.5 * (a - d);
        fail = p * p + bq * e < 0.0 ? kGeComplex : kGeNoConv;
        break;
      }
      // shift: the eigenvalue of the trailing 2 x 2 block nearer its last
      // diagonal entry (Wilkinson), its last diagonal entry when that block has
      // complex eigenvalues, and an ad hoc exceptional shift every 10th step
      const double a = uni(H[pk(hi - 1, hi - 1)]), bq = uni(H[pk(hi - 1, hi)]);
      const double e = uni(H[pk(hi, hi - 1)]), d = uni(H[pk(hi, hi)]);
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
      // bulge chased down the window.  Rotation k turns rows (k, k+1) (lane =
      // column, columns j0..n-1) and then columns (k, k+1) (lane = row, rows
      // 0..i1).  Every lane also carries the entries the chain needs next: the
      // 2 x 2 window H[k..k+1, k..k+1] and H[k+2, k+1] before rotation k, from
      // which the pair (h_{k+1,k}, h_{k+2,k}) of rotation k+1 follows with the
      // operations the updating lanes apply (so the copies equal the stored
      // entries, up to the sign of a zero).  The rotation of step k+1 is thus
      // formed while the lanes update the matrix for step k, and the LDS carries
      // no value of the chain.  Lanes outside a rotation's range store into J
      // instead of being masked, which keeps the step one straight block of code.
      const int lr = l < NM ? l : NM - 1;
      double c, s;
      givens_chase(uni(H[pk(lo, lo)]) - sigma, uni(H[pk(lo + 1, lo)]), c, s);
      double wa = uni(H[pk(lo, lo)]), wb = uni(H[pk(lo, lo + 1)]);
      double wd = uni(H[pk(lo + 1, lo)]), we = uni(H[pk(lo + 1, lo + 1)]);
      double wf = uni(H[pk(lo + 2, lo + 1)]);  // lo + 2 <= hi: the window has three rows at least
      compiler_fence();
#pragma unroll 2
      for (int k = lo; k < hi; ++k) {
        const int j0 = k > lo ? k - 1 : lo;
        const int i1 = k + 2 < hi ? k + 2 : hi;
        // rows k, k+1 of this lane's column (outside the packed column for
        // lanes left of j0: read, never stored), and column k+2 rows k..k+3 (the
        // window of rotation k+1; clamped into H on the last step, unused there)
        const lds_t<double>* rp = H + pk(k, lr);
        const double ra = rp[0], rb = rp[1];
        const int wo = min(pk(k, k + 2), PS - 4);
        const double g0 = H[wo], g1 = H[wo + 1], g2 = H[wo + 2], g3 = H[wo + 3];
        // the chain: rotation k on the window, then rotation k+1
        const double d1 = rot_lo(c, s, wa, wd), e1 = rot_lo(c, s, wb, we);
        const double xn = rot_hi(c, s, d1, e1), an = rot_lo(c, s, d1, e1);
        const double yn = s * wf, dn = c * wf;
        double cn, sn;
        givens_chase(xn, yn, cn, sn);
        // rows k, k+1; the bulge h_{k+1,k-1} is annihilated exactly
        const double ra2 = rot_hi(c, s, ra, rb);
        const double rb2 = l == k - 1 ? 0.0 : rot_lo(c, s, ra, rb);
        lds_t<double>* rw = (l >= j0 && l < n) ? H + pk(k, l) : J + 2 * l;
        rw[0] = ra2;
        rw[1] = rb2;
        // columns k, k+1 (k + 3 apart in the packed layout), read after the row update
        const lds_t<double>* cp = H + pk(lr, k);
        const double ca = cp[0], cb = cp[k + 3];
        lds_t<double>* cw = l <= i1 ? H + pk(l, k) : J + l;
        cw[0] = rot_hi(c, s, ca, cb);
        cw[k + 3] = rot_lo(c, s, ca, cb);
        lds_t<double>* sw = l == 0 ? cs + 2 * k : J + 2 * l;
        sw[0] = c;
        sw[1] = s;
        // the window of rotation k+1
        wb = rot_lo(c, s, g0, g1);
        wa = an;
        wd = dn;
        we = g2;
        wf = g3;
        c = cn;
        s = sn;
      }
      rlo = lo;
      rhi = hi;
    }
    // one place applies the step's rotations to the Schur vectors
    if (rhi > rlo) {
      compiler_fence();
      rotate_q<NM>(q, cs, rlo, rhi);
      compiler_fence();
      reset_rotations(cs, rlo, rhi);
    }
  }
  if (fail != 0) {
    if (l == 0) S.status[b] = fail;
    return;
  }
  // ---- egress: T (or T^T) with exact zeros off its triangle, scaled back, and Q
  for (int j = 0; j < n; ++j) {
    if (l < n) {
      double v;
      if (S.lower) v = l >= j ? H[pk(j, l)] : 0.0;
      else v = l <= j ? H[pk(l, j)] : 0.0;
      T[l + (size_t)j * ld] = ldexp(v, esc);
    }
  }
  // in descending order, columns past n-1 clamped onto column n-1: its own
  // value is stored last (same lane, same address)
  if (l < n) {
    gbl_t<double>* Qp = Q + l;
#pragma unroll
    for (int j = NM - 1; j >= 0; --j) Qp[(size_t)(j < n ? j : n - 1) * ld] = q[j];
  }
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
  L.bytes = L.int_off + (size_t)8 * batch * sizeof(int);
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
  int* esc0 = ints + 6 * batch;
  int* esc1 = ints + 7 * batch;

  SchurArgs sa{};
  sa.batch = batch;
  sa.n_max = nm;
  sa.nsets = syl ? 2 : 1;
  sa.n = n;
  sa.stride = Lo.stride;
  sa.set[0] = SchurSet{A, lda, 1, 1, Lt, Zq, st0, esc0};
  if (syl) sa.set[1] = SchurSet{B, ldb, 0, 0, Ut, Wq, st1, esc1};
  const dim3 sg(batch * sa.nsets);
  if (nm <= 16) {
    hipLaunchKernelGGL((k_hess<16, 1>), sg, dim3(64), 0, h->stream, sa);
    hipLaunchKernelGGL(k_schur_qr<16>, sg, dim3(64), 0, h->stream, sa);
  } else if (nm <= 32) {
    hipLaunchKernelGGL((k_hess<32, 1>), sg, dim3(64), 0, h->stream, sa);
    hipLaunchKernelGGL(k_schur_qr<32>, sg, dim3(64), 0, h->stream, sa);
  } else {
    hipLaunchKernelGGL((k_hess<64, 2>), sg, dim3(128), 0, h->stream, sa);
    hipLaunchKernelGGL(k_schur_qr<64>, sg, dim3(64), 0, h->stream, sa);
  }
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
