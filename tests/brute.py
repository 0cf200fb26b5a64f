"""Brute-force numerical integrals used to pin the oracle.

Independent of the Boys function and of McMurchie-Davidson: the Coulomb
kernel is written as 1/r = (2/sqrt(pi)) int_0^inf exp(-t^2 r^2) dt, each
Cartesian direction then becomes a two-dimensional Gaussian integral that a
tensor Gauss-Hermite rule integrates exactly after the quadratic form is
diagonalised, and the t integral is done by composite Gauss-Legendre after
mapping [0, inf) to [0, 1).  Angular shapes come from the input generator's
own shape functions (fitted to monomials), normalised numerically.
"""
import itertools
import math

import numpy as np

from workload.water import _shapes

_GH_T, _GH_W = np.polynomial.hermite.hermgauss(8)


def monomials(l):
    return [(lx, ly, l - lx - ly) for lx in range(l, -1, -1) for ly in range(l - lx, -1, -1)]


def shape_coefficients(l):
    """(2l+1, ncart) monomial coefficients of the generator's shapes."""
    rng = np.random.default_rng(7)
    pts = rng.standard_normal((64, 3))
    mons = monomials(l)
    A = np.array([[x ** a * y ** b * z ** c for (a, b, c) in mons] for x, y, z in pts])
    out = []
    for f in _shapes(l, pts[:, 0], pts[:, 1], pts[:, 2]):
        coef, *_ = np.linalg.lstsq(A, f * np.ones(len(pts)), rcond=None)
        out.append(coef)
    return np.array(out)


def _gauss_moment(n, beta):
    """int x^n exp(-beta x^2) dx over the real line."""
    if n % 2:
        return 0.0
    return math.gamma((n + 1) / 2) / beta ** ((n + 1) / 2)


def sph_norms(l, a):
    """Numerical normalisation of each shape function with exponent a."""
    cf = shape_coefficients(l)
    mons = monomials(l)
    out = []
    for m in range(2 * l + 1):
        s = 0.0
        for i, mi in enumerate(mons):
            for j, mj in enumerate(mons):
                s += cf[m, i] * cf[m, j] * np.prod([_gauss_moment(mi[d] + mj[d], 2 * a) for d in range(3)])
        out.append(1.0 / math.sqrt(s))
    return np.array(out)


def _t_rule(npanel=24, order=24):
    """Nodes/weights for int_0^inf g(t) dt with t = s/(1-s)."""
    x, w = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(0.0, 1.0, npanel + 1) ** 1.5
    S, Wt = [], []
    for a, b in zip(edges[:-1], edges[1:]):
        S.append(0.5 * (b - a) * x + 0.5 * (b + a))
        Wt.append(0.5 * (b - a) * w)
    s = np.concatenate(S)
    ws = np.concatenate(Wt)
    t = s / (1.0 - s)
    return t, ws / (1.0 - s) ** 2


_T, _TW = _t_rule()


def _dir_integrals(exps, cents, lmax, t):
    """Per-direction 2-D integrals for a bra pair (a@A, b@B) and ket (g@C):
    out[i][j][k][tidx] = int int (x1-A)^i (x1-B)^j (x2-C)^k
                         exp(-a(x1-A)^2 - b(x1-B)^2 - g(x2-C)^2 - t^2 (x1-x2)^2)."""
    a, b, g = exps
    A, B, C = cents
    la, lb, lc = lmax
    t2 = t * t
    nt = len(t)
    M = np.zeros((nt, 2, 2))
    M[:, 0, 0] = a + b + t2
    M[:, 0, 1] = M[:, 1, 0] = -t2
    M[:, 1, 1] = g + t2
    h = np.array([a * A + b * B, g * C])
    Minv = np.linalg.inv(M)
    xs = Minv @ h                                    # (nt, 2) centres
    const = a * A * A + b * B * B + g * C * C - np.einsum("i,tij,j->t", h, Minv, h)
    G = np.linalg.cholesky(M)                        # M = G G^T
    Ginv_T = np.linalg.inv(np.transpose(G, (0, 2, 1)))
    det = G[:, 0, 0] * G[:, 1, 1]
    y1, y2 = np.meshgrid(_GH_T, _GH_T, indexing="ij")
    wy = np.outer(_GH_W, _GH_W).ravel()
    Y = np.stack([y1.ravel(), y2.ravel()])           # (2, nq)
    X = xs[:, :, None] + Ginv_T @ Y[None]            # (nt, 2, nq)
    x1, x2 = X[:, 0, :], X[:, 1, :]
    base = np.exp(-const)[:, None] / det[:, None] * wy[None, :]
    out = np.zeros((la + 1, lb + 1, lc + 1, nt))
    for i in range(la + 1):
        for j in range(lb + 1):
            for k in range(lc + 1):
                out[i, j, k] = np.sum(base * (x1 - A) ** i * (x1 - B) ** j * (x2 - C) ** k, axis=1)
    return out


def coulomb3c_block(la, a, A, lb, b, B, lc, g, C):
    """(ab|c) spherical block (2la+1, 2lb+1, 2lc+1) of unit-normalised functions."""
    A, B, C = (np.asarray(v, float) for v in (A, B, C))
    per_dir = [_dir_integrals((a, b, g), (A[d], B[d], C[d]), (la, lb, lc), _T) for d in range(3)]
    ma, mb, mc = monomials(la), monomials(lb), monomials(lc)
    cart = np.zeros((len(ma), len(mb), len(mc)))
    for (ia, ea), (ib, eb), (ic, ec) in itertools.product(enumerate(ma), enumerate(mb), enumerate(mc)):
        f = per_dir[0][ea[0], eb[0], ec[0]] * per_dir[1][ea[1], eb[1], ec[1]] * per_dir[2][ea[2], eb[2], ec[2]]
        cart[ia, ib, ic] = 2.0 / math.sqrt(math.pi) * np.sum(f * _TW)
    ca = shape_coefficients(la) * sph_norms(la, a)[:, None]
    cb = shape_coefficients(lb) * sph_norms(lb, b)[:, None]
    cc = shape_coefficients(lc) * sph_norms(lc, g)[:, None]
    return np.einsum("xi,yj,zk,ijk->xyz", ca, cb, cc, cart)


def boys0(T):
    if T < 1e-15:
        return 1.0
    return 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))


def ssss(a, A, b, B, c, C, d, D):
    """Closed-form (ab|cd) over four normalised s Gaussians."""
    A, B, C, D = (np.asarray(v, float) for v in (A, B, C, D))
    n = lambda e: (2 * e / math.pi) ** 0.75
    p, q = a + b, c + d
    P = (a * A + b * B) / p
    Q = (c * C + d * D) / q
    kab = math.exp(-a * b / p * np.sum((A - B) ** 2))
    kcd = math.exp(-c * d / q * np.sum((C - D) ** 2))
    al = p * q / (p + q)
    return (n(a) * n(b) * n(c) * n(d) * 2 * math.pi ** 2.5 / (p * q * math.sqrt(p + q))
            * kab * kcd * boys0(al * np.sum((P - Q) ** 2)))


def _dir_integrals4(exps, cents, lmax, t):
    """Per-direction 2-D integrals for a bra pair (a@A, b@B) and a ket pair
    (c@C, d@D): out[i][j][k][l][tidx] = int int (x1-A)^i (x1-B)^j (x2-C)^k (x2-D)^l
    exp(-a(x1-A)^2 - b(x1-B)^2 - c(x2-C)^2 - d(x2-D)^2 - t^2 (x1-x2)^2)."""
    a, b, c, d = exps
    A, B, C, D = cents
    la, lb, lc, ld = lmax
    t2 = t * t
    nt = len(t)
    M = np.zeros((nt, 2, 2))
    M[:, 0, 0] = a + b + t2
    M[:, 0, 1] = M[:, 1, 0] = -t2
    M[:, 1, 1] = c + d + t2
    h = np.array([a * A + b * B, c * C + d * D])
    Minv = np.linalg.inv(M)
    xs = Minv @ h
    const = a * A * A + b * B * B + c * C * C + d * D * D - np.einsum("i,tij,j->t", h, Minv, h)
    G = np.linalg.cholesky(M)
    Ginv_T = np.linalg.inv(np.transpose(G, (0, 2, 1)))
    det = G[:, 0, 0] * G[:, 1, 1]
    y1, y2 = np.meshgrid(_GH_T, _GH_T, indexing="ij")
    wy = np.outer(_GH_W, _GH_W).ravel()
    Y = np.stack([y1.ravel(), y2.ravel()])
    X = xs[:, :, None] + Ginv_T @ Y[None]
    x1, x2 = X[:, 0, :], X[:, 1, :]
    base = np.exp(-const)[:, None] / det[:, None] * wy[None, :]
    out = np.zeros((la + 1, lb + 1, lc + 1, ld + 1, nt))
    for i, j, k, l in itertools.product(range(la + 1), range(lb + 1), range(lc + 1), range(ld + 1)):
        out[i, j, k, l] = np.sum(base * (x1 - A) ** i * (x1 - B) ** j * (x2 - C) ** k * (x2 - D) ** l, axis=1)
    return out


def coulomb4c_block(la, a, A, lb, b, B, lc, c, C, ld, d, D):
    """(ab|cd) spherical block (2la+1, 2lb+1, 2lc+1, 2ld+1) of unit-normalised functions."""
    A, B, C, D = (np.asarray(v, float) for v in (A, B, C, D))
    per_dir = [_dir_integrals4((a, b, c, d), (A[x], B[x], C[x], D[x]), (la, lb, lc, ld), _T) for x in range(3)]
    ms = [monomials(l) for l in (la, lb, lc, ld)]
    cart = np.zeros(tuple(len(m) for m in ms))
    for idx in itertools.product(*[range(len(m)) for m in ms]):
        e = [ms[k][idx[k]] for k in range(4)]
        f = np.ones_like(_T)
        for x in range(3):
            f = f * per_dir[x][e[0][x], e[1][x], e[2][x], e[3][x]]
        cart[idx] = 2.0 / math.sqrt(math.pi) * np.sum(f * _TW)
    cs = [shape_coefficients(l) * sph_norms(l, g)[:, None] for l, g in ((la, a), (lb, b), (lc, c), (ld, d))]
    return np.einsum("wi,xj,yk,zl,ijkl->wxyz", *cs, cart)
