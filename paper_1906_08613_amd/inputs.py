"""Seeded synthetic inputs for the batched solvers.

This module holds no arithmetic of the solvers themselves: it only draws
random matrices with the structure each operation expects (symmetric positive
definite A, lower/upper triangular L/U, symmetric S) and is the one piece of
code shared by the tests, the benchmark and the oracle checks, so that both
sides of every comparison see identical bytes.

Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used as a counter-based
generator: draw k of stream s is mix(s + (k+1)*gamma).  Uniforms take the top
53 bits; normals use the Box-Muller transform.

Every instance has its own stream, seeded by a 64-bit hash of
(workload tag, op, n, kappa, instance index), so any subset of a batch can be
regenerated on its own.

Matrices are returned as numpy arrays of shape (batch, n, n) indexed [b, i, j].
"""
from __future__ import annotations

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)
_MASK = (1 << 64) - 1


def _mix(z):
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def splitmix64(seeds, count):
    """uint64 array (len(seeds), count): draw k of stream s is mix(s + (k+1) gamma)."""
    seeds = np.asarray(seeds, dtype=np.uint64).reshape(-1, 1)
    k = np.arange(1, count + 1, dtype=np.uint64).reshape(1, -1)
    with np.errstate(over="ignore"):
        return _mix(seeds + k * _GAMMA)


def uniform(seeds, count):
    """U[0,1) doubles from the top 53 bits."""
    return (splitmix64(seeds, count) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def normal(seeds, count):
    """N(0,1) by Box-Muller on consecutive uniform pairs."""
    m = (count + 1) // 2
    u = uniform(seeds, 2 * m)
    u1 = 1.0 - u[:, 0::2]          # (0, 1]
    u2 = u[:, 1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)], axis=1)
    return z[:, :count]


_OPS = {"potrf": 1, "trsyl": 2, "trlyap": 3, "ragged": 4, "mlp": 5, "gesyl": 8, "gelyap": 9}


def instance_seeds(tag, op, n, kappa, batch, start=0):
    """Per-instance 64-bit seeds: hash of (tag, op, n, kappa, instance)."""
    key = (hash_str(tag) * 0x100000001B3) & _MASK
    key ^= _OPS.get(op, 7) * 0xD6E8FEB86659FD93
    key ^= (int(n) * 0xFF51AFD7ED558CCD) & _MASK
    key ^= int(np.float64(kappa).view(np.uint64)) * 0xC4CEB9FE1A85EC53 & _MASK
    key &= _MASK
    idx = np.arange(start, start + batch, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(np.uint64(key) ^ _mix(idx + _GAMMA))


def hash_str(s: str) -> int:
    """FNV-1a 64-bit of a string."""
    h = 0xCBF29CE484222325
    for ch in s.encode():
        h ^= ch
        h = (h * 0x100000001B3) & _MASK
    return h


# ---------------------------------------------------------------- workloads
def spd_shifted(seeds, n):
    """A = B^T B + n I with B i.i.d. uniform[-1, 1] (Cholesky workloads)."""
    b = len(seeds)
    B = 2.0 * uniform(seeds, n * n).reshape(b, n, n) - 1.0
    A = np.matmul(np.swapaxes(B, 1, 2), B)
    A[:, np.arange(n), np.arange(n)] += n
    return 0.5 * (A + np.swapaxes(A, 1, 2))


def triangular(seeds, n, lower=True, diag_lo=1.0, diag_hi=2.0, off_scale=None):
    """Triangular matrix: off-diagonal N(0,1)*off_scale (default 1/n), diagonal U[lo, hi]."""
    b = len(seeds)
    if off_scale is None:
        off_scale = 1.0 / max(n, 1)
    z = normal(seeds, n * n).reshape(b, n, n) * off_scale
    d = diag_lo + (diag_hi - diag_lo) * uniform(seeds ^ np.uint64(0xA5A5A5A5A5A5A5A5), n)
    T = np.tril(z, -1) if lower else np.triu(z, 1)
    T[:, np.arange(n), np.arange(n)] = d
    return T


def gaussian(seeds, n):
    """Dense N(0,1) n x n matrices."""
    return normal(seeds, n * n).reshape(len(seeds), n, n)


def symmetric(seeds, n):
    """Symmetric matrices: lower triangle N(0,1), mirrored."""
    Z = gaussian(seeds, n)
    low = np.tril(Z)
    return low + np.swapaxes(np.tril(Z, -1), 1, 2)


def _sub(seeds, k):
    with np.errstate(over="ignore"):
        return _mix(seeds + np.uint64(0x632BE59BD9B4E019) * np.uint64(k + 1))


def potrf_problem(tag, n, batch, start=0):
    s = instance_seeds(tag, "potrf", n, 0.0, batch, start)
    return spd_shifted(s, n)


def trsyl_problem(tag, n, batch, start=0):
    """L lower / U upper: off-diagonal N(0,1)/n, diagonal U[1,2]; C ~ N(0,1)."""
    s = instance_seeds(tag, "trsyl", n, 0.0, batch, start)
    L = triangular(_sub(s, 0), n, lower=True)
    U = triangular(_sub(s, 1), n, lower=False)
    C = gaussian(_sub(s, 2), n)
    return L, U, C


def trlyap_problem(tag, n, batch, start=0):
    """L lower as for trsyl; S symmetric N(0,1)."""
    s = instance_seeds(tag, "trlyap", n, 0.0, batch, start)
    L = triangular(_sub(s, 0), n, lower=True)
    S = symmetric(_sub(s, 1), n)
    return L, S


# ------------------------------------------------ condition-controlled inputs
def haar_orthogonal(seeds, n):
    """Haar-distributed orthogonal Q: QR of a Gaussian with diag(R) made positive."""
    G = gaussian(seeds, n)
    Q, R = np.linalg.qr(G)
    sgn = np.sign(np.diagonal(R, axis1=1, axis2=2))
    sgn[sgn == 0] = 1.0
    return Q * sgn[:, None, :]


def potrf_kappa(tag, n, batch, kappa, start=0):
    """A = Q diag(sigma) Q^T with sigma_i = kappa^(-i/(n-1)): 2-norm condition kappa."""
    s = instance_seeds(tag, "potrf", n, kappa, batch, start)
    Q = haar_orthogonal(s, n)
    if n > 1:
        sig = kappa ** (-np.arange(n) / (n - 1))
    else:
        sig = np.ones(1)
    A = np.matmul(Q * sig[None, None, :], np.swapaxes(Q, 1, 2))
    return 0.5 * (A + np.swapaxes(A, 1, 2))


def _geom_diag(seeds, n, kappa):
    """Shuffled geometric sequence on [1/kappa, 1] per instance."""
    b = len(seeds)
    base = kappa ** (-np.arange(n) / max(n - 1, 1))
    keys = uniform(seeds, n)
    order = np.argsort(keys, axis=1, kind="stable")
    return np.broadcast_to(base, (b, n))[np.arange(b)[:, None], order]


def _tri_kappa(seeds, n, kappa, lower):
    b = len(seeds)
    dmin = 1.0 / kappa
    z = normal(seeds, n * n).reshape(b, n, n) * (dmin / max(n, 1))
    T = np.tril(z, -1) if lower else np.triu(z, 1)
    T[:, np.arange(n), np.arange(n)] = _geom_diag(_sub(seeds, 9), n, kappa)
    return T


def trsyl_kappa(tag, n, batch, kappa, start=0):
    """Diagonals geometric on [1/kappa, 1] (shuffled), off-diagonals N(0,1)/(kappa n), C ~ N(0,1)."""
    s = instance_seeds(tag, "trsyl", n, kappa, batch, start)
    L = _tri_kappa(_sub(s, 0), n, kappa, True)
    U = _tri_kappa(_sub(s, 1), n, kappa, False)
    C = gaussian(_sub(s, 2), n)
    return L, U, C


def trlyap_kappa(tag, n, batch, kappa, start=0):
    s = instance_seeds(tag, "trlyap", n, kappa, batch, start)
    L = _tri_kappa(_sub(s, 0), n, kappa, True)
    S = symmetric(_sub(s, 1), n)
    return L, S


# --------------------------------------------------------------- ragged mix
def ragged_mix(tag, batch, n_lo=3, n_hi=128, fractions=(0.4, 0.3, 0.3)):
    """Ops and sizes of a ragged batch: op drawn with the given fractions, n uniform on {n_lo..n_hi}."""
    s = instance_seeds(tag, "ragged", 0, 0.0, batch)
    u = uniform(s, 2)
    c = np.cumsum(fractions)
    ops = np.searchsorted(c / c[-1], u[:, 0], side="right").astype(np.int32)
    ops = np.minimum(ops, 2)
    ns = (n_lo + np.floor(u[:, 1] * (n_hi - n_lo + 1))).astype(np.int32)
    return ops, np.minimum(ns, n_hi)


# ------------------------------------------------ general (non-triangular) coefficients
def real_spectrum(seeds, n, lo=1.0, hi=2.0, off_scale=None):
    """M = Q T Q^T: Q Haar orthogonal, T upper triangular with diagonal U[lo, hi]
    and strictly upper part N(0,1) * off_scale (default 1/n); a non-normal
    matrix whose eigenvalues are T's diagonal (all real).  The 1/n scale keeps
    the eigenvalues well conditioned (condition numbers up to about 1e5 at
    n = 64); at 1/sqrt(n) random triangular matrices grow exponentially
    ill-conditioned eigenvalues, and close pairs turn into complex pairs
    once M is rounded to FP64."""
    if off_scale is None:
        off_scale = 1.0 / max(n, 1)
    T = triangular(_sub(seeds, 10), n, lower=False, diag_lo=lo, diag_hi=hi, off_scale=off_scale)
    # stratified eigenvalues: one in each of n equal slots of [lo, hi] (kept
    # off the slot edges), in random order, so that no two are closer than
    # (hi - lo) / (2 n); independent uniform draws put close pairs into a few
    # instances per thousand, which rounding turns into complex pairs
    u = uniform(_sub(seeds, 12), 2 * n).reshape(len(seeds), 2, n)
    slot = np.argsort(u[:, 0, :], axis=1)
    T[:, np.arange(n), np.arange(n)] = lo + (hi - lo) * (slot + 0.25 + 0.5 * u[:, 1, :]) / max(n, 1)
    Q = haar_orthogonal(_sub(seeds, 11), n)
    return np.matmul(np.matmul(Q, T), np.swapaxes(Q, 1, 2))


def gesyl_problem(tag, n, batch, start=0):
    """A, B with real spectra in [1, 2] (so every lambda_i(A) + lambda_j(B) >= 2); C ~ N(0,1)."""
    s = instance_seeds(tag, "gesyl", n, 0.0, batch, start)
    A = real_spectrum(_sub(s, 0), n)
    B = real_spectrum(_sub(s, 1), n)
    C = gaussian(_sub(s, 2), n)
    return A, B, C


def gelyap_problem(tag, n, batch, start=0):
    """Stable A with real spectrum in [-2, -1]; S symmetric N(0,1)."""
    s = instance_seeds(tag, "gelyap", n, 0.0, batch, start)
    A = real_spectrum(_sub(s, 0), n, lo=-2.0, hi=-1.0)
    S = symmetric(_sub(s, 1), n)
    return A, S

