"""Reference evaluations of the lower-precision formats of the K contraction
(test infrastructure; only tests, the smoke check and the benchmark's CPU leg
use this module).

K = 2 X X^T, X_{mu k} the half-transformed tensor with k = (P, i).  Each
function below takes X (FP64, from the oracle) to the number format a mixed
build stores it in and evaluates the products that format keeps in exact
arithmetic, so a device result can be compared with the format itself (its
rounding of the sums is then the only difference) and with the FP64 oracle
(the format's own error).  The paper proposes single precision for later
SCF iterations (Section 5, "Limitations and Future Development: Mixed
Precision") without fixing a format; the three formats are this project's:

* FP32: X rounded to binary32 (round to nearest even).
* BF16x3: the binary32 value split into hi = bf16(x32) and lo = bf16(x32 - hi)
  (round to nearest even); products hi.hi + hi.lo + lo.hi.
* INT8 (Ozaki et al., Numer. Algorithms 59, 2012): blocks of `block`
  consecutive k of one row share a power-of-two scale 2^e, e the least
  integer with 2^e > max|x| 128/127; x 2^-e = sum_{s<n} a_s 2^{-7(s+1)}
  + r by repeated rounding to nearest even (t <- 128 t, a_s = rint(t),
  t <- t - a_s), so a_0 in [-127, 127], a_s in [-64, 64] for s >= 1 and
  |r| <= 2^{-7n-1}; products a_i b_j of order i + j <= n - 1 are kept.
"""
from __future__ import annotations

import numpy as np


def round_fp32(X):
    """X rounded to binary32 and back (the FP32 storage of X)."""
    return np.asarray(X, np.float64).astype(np.float32).astype(np.float64)


def _bf16(x32):
    """binary32 -> bfloat16 by round to nearest even, returned as float64."""
    u = np.ascontiguousarray(x32, np.float32).view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def split_bf16(X):
    """(hi, lo): hi = bf16(x32), lo = bf16(x32 - hi), x32 = fp32(x)."""
    x32 = np.asarray(X, np.float64).astype(np.float32)
    hi = _bf16(x32)
    lo = _bf16((x32.astype(np.float64) - hi).astype(np.float32))
    return hi, lo


def int8_slices(X, block=256, nslices=5):
    """Slices of every row of X (n x kdim, kdim a multiple of block).
    Returns (a, e): a[s] integer-valued float64 arrays (n x kdim) and the
    block exponents e (n x kdim/block)."""
    X = np.asarray(X, np.float64)
    n, kdim = X.shape
    if kdim % block:
        raise ValueError("kdim must be a multiple of the block")
    Xb = X.reshape(n, kdim // block, block)
    m = np.abs(Xb).max(axis=2)
    e = np.where(m > 0, np.frexp(m * (128.0 / 127.0))[1], 0).astype(np.int64)
    t = np.ldexp(Xb, -e[:, :, None])
    a = []
    for _ in range(nslices):
        t = t * 128.0
        s = np.rint(t)
        t = t - s
        a.append(s.reshape(n, kdim))
    return a, e


def int8_product(A, B, block=256, nslices=5, keep=None):
    """sum_k x_{mu k} y_{nu k} for the int8 slices of the rows of A and B,
    with the products a_i b_j of order i + j <= nslices - 1 (or those for
    which keep(i, j) is true) summed exactly per block and scaled by
    2^{e_mu + e_nu} per block, accumulated in FP64."""
    if keep is None:
        def keep(i, j):
            return i + j <= nslices - 1
    a, ea = int8_slices(A, block, nslices)
    b, eb = int8_slices(B, block, nslices)
    nb = ea.shape[1]
    out = np.zeros((A.shape[0], B.shape[0]))
    for blk in range(nb):
        sl = slice(blk * block, (blk + 1) * block)
        acc = np.zeros_like(out)
        for i in range(nslices):
            for j in range(nslices):
                if keep(i, j):
                    # integers below 2^53: the float64 matrix product is exact
                    acc += np.ldexp(a[i][:, sl] @ b[j][:, sl].T, -7 * (i + j + 2))
        out += acc * np.ldexp(1.0, ea[:, blk][:, None] + eb[:, blk][None, :])
    return out


def int8_fast_keep(i, j):
    """The products of the four-order variant: i + j <= 3, and a_2 b_2 (a
    square on the diagonal of K, so the one order-4 product whose omission
    would bias E_K)."""
    return i + j <= 3 or (i, j) == (2, 2)


def int8_scale_envelope(A, B, block=256, nslices=5):
    """S_{mu nu} = sum_k 2^{e_mu(k) + e_nu(k)}: times 2^-33 it bounds the
    truncation error of int8_product (each kept-set product is within
    2^{-7n+2} 2^{e_x + e_y} of x y for n = 5 slices: the dropped orders sum
    to under 1.01 2^-35 and the remainders to 2^-35)."""
    def scales(X):
        X = np.asarray(X, np.float64)
        m = np.abs(X.reshape(X.shape[0], -1, block)).max(axis=2)
        _, e = int8_slices(X, block, nslices)
        return np.where(m > 0, np.ldexp(1.0, e), 0.0)   # an all-zero block is exact
    return block * (scales(A) @ scales(B).T)


def gram_lambda_bound(C, squarings=4):
    """An upper bound of lambda_max(C^T C): |(C^T C)^(2^s)|_F^(2^-s), each
    square normalised by its Frobenius norm (the Frobenius norm bounds the
    spectral one)."""
    M = np.asarray(C, np.float64).T @ np.asarray(C, np.float64)
    f0 = np.linalg.norm(M)
    if f0 == 0.0:
        return 0.0, 0.0
    P = M / f0
    log_l = np.log(f0)
    for t in range(1, squarings + 1):
        P = P @ P
        g = np.linalg.norm(P)
        P = P / g
        log_l += np.log(g) / 2 ** t
    return f0, np.exp(log_l)


def int8_energy_bound(A, C, EK_int8, nsums, block=256):
    """Bound on |E_K(int8) - E_K(exact)| for K = 2 A A^T (rows A[mu], k),
    E_K = -1/4 Tr(D K), D = 2 C C^T, by Cauchy-Schwarz in the D-seminorm:
      1/2 [2 sqrt(Q lam R) + lam R + lam T] + F
    with A_s the sums of squares of the scaled digits, R the remainders'
    block-scale bound, T = sum_{i+j>=5} sqrt(A_i A_j), lam >= lambda_max(D),
    Q = 2 |E_K(int8)| + lam T + 2F, F the FP64 fold rounding (nsums sums).
    Returns a dict with the bound and its parts."""
    A = np.asarray(A, np.float64)
    n, kdim = A.shape
    a, e = int8_slices(A, block)
    E = np.repeat(e, block, axis=1)
    As = [float((np.ldexp(a[s], E - 7 * (s + 1)) ** 2).sum()) for s in range(len(a))]
    R = float((256.0 * np.ldexp(1.0, 2 * e - 72)).sum())
    ns = len(a)
    T = sum(np.sqrt(As[i] * As[j]) for i in range(1, ns) for j in range(1, ns) if i + j >= ns)
    f0, lmax = gram_lambda_bound(C)
    lam = 2.0 * lmax
    u = 2.0 ** -53
    F = nsums * u / (1 - nsums * u) * 2.0 * f0 * sum(np.sqrt(x) for x in As) ** 2
    Q = 2.0 * abs(EK_int8) + lam * T + 2.0 * F
    bound = 0.5 * (2.0 * np.sqrt(Q * lam * R) + lam * R + lam * T) + F
    return dict(bound=bound, lam=lam, R=R, T=T, Q=Q, A=As, F=F)
