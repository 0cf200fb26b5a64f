"""FP64 CPU oracle for the density-fitted J/K build (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this package.  It shares no code with the GPU library.  The integrals, the
Boys function, the Cholesky factor and the forward substitution live in the
plain C file ``oracle.c``; this module strings them together with numpy in
the order the textbook definition of Coulomb-metric density fitting gives:

    U_{P,mu nu} = (mu nu | P)                 three-centre integrals
    V_{PQ}      = (P | Q),  V = L L^T          metric and its Cholesky factor
    B           = L^{-1} U                     whitened three-centre tensor
    c_P         = sum_{mu nu} B_{P,mu nu} D_{mu nu}
    J_{mu nu}   = sum_P B_{P,mu nu} c_P
    K_{mu nu}   = sum_P sum_{la si} B_{P,mu la} D_{la si} B_{P,si nu}
    E_J = 1/2 Tr(D J),   E_K = -1/4 Tr(D K)

With occupied orbitals C the density is D = 2 C C^T (closed shell) and K is
taken through the half-transformed tensor X_{P,mu i} = sum_nu B_{P,mu nu} C_{nu i},
K = 2 sum_{P,i} X_{P,mu i} X_{P,nu i}.  None of these formulas appears in the
paper (GPU4PySCF v1.0), which only names the method (Introduction; Section
"Dataset and Performance"); they are the standard Coulomb-metric fitting
(Whitten 1973; Vahtras, Almloef and Feyereisen 1993).

For the four-centre direct path (the direct-SCF J/K that the paper's
package started from, Introduction; "Limitations and Future Development:
Direct SCF & Other Integral Schemes") the oracle gives the
unfitted definitions J_{mu nu} = sum (mu nu|la si) D_{la si} and
K_{mu nu} = sum (mu la|nu si) D_{la si}: dense for tiny systems
(``exact_jk``) and one shell-pair block at a time for large ones
(``exact_jk_blocks``), both unscreened.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    """Load (building if needed) the C oracle."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB) or (
                os.path.getmtime(_build.LIB) < os.path.getmtime(os.path.join(_build.HERE, "oracle.c"))):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        dp = ctypes.POINTER(ctypes.c_double)
        ip = ctypes.POINTER(ctypes.c_int)
        L.orc_boys.argtypes = [ctypes.c_int, ctypes.c_double, dp]
        L.orc_norm.argtypes = [ctypes.c_int, ctypes.c_double]
        L.orc_norm.restype = ctypes.c_double
        L.orc_int3c.argtypes = [dp, ctypes.c_int, ip, ip, dp, ctypes.c_int, ip, ip, dp,
                                ctypes.c_int, ctypes.c_int, dp]
        L.orc_int2c.argtypes = [dp, ctypes.c_int, ip, ip, dp, dp]
        L.orc_int4c.argtypes = [dp, ctypes.c_int, ip, ip, dp, dp]
        L.orc_jk_blocks.argtypes = [dp, ctypes.c_int, ip, ip, dp, dp, ctypes.c_int, ip, ip,
                                    ctypes.POINTER(ctypes.c_long), dp, dp]
        L.orc_overlap.argtypes = [dp, ctypes.c_int, ip, ip, dp, dp]
        L.orc_cholesky.argtypes = [ctypes.c_long, dp, dp]
        L.orc_cholesky.restype = ctypes.c_long
        L.orc_forward_subst.argtypes = [ctypes.c_long, dp, ctypes.c_long, dp]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _d(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _i(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int))


def _basis(atom, l, e):
    return (len(l), np.ascontiguousarray(atom, np.int32), np.ascontiguousarray(l, np.int32),
            np.ascontiguousarray(e, np.float64))


def num_threads():
    return lib().orc_num_threads()


def boys(mmax, T):
    """F_0(T) .. F_mmax(T)."""
    F = np.zeros(mmax + 1)
    lib().orc_boys(mmax, float(T), _d(F))
    return F


def norm(l, a):
    """Normalisation constant N_l(a) of a Racah-normalised solid-harmonic Gaussian."""
    return lib().orc_norm(l, float(a))


def int3c(mol, c0=0, c1=None):
    """(mu nu|P) for aux shells [c0, c1): array (naux_slice, nao, nao)."""
    n, aa, al, ae = _basis(mol.ao_atom, mol.ao_l, mol.ao_exp)
    m, xa, xl, xe = _basis(mol.aux_atom, mol.aux_l, mol.aux_exp)
    if c1 is None:
        c1 = m
    nsl = int(np.sum(2 * xl[c0:c1] + 1))
    out = np.zeros((nsl, mol.nao, mol.nao))
    xyz = np.ascontiguousarray(mol.coords, np.float64)
    rc = lib().orc_int3c(_d(xyz), n, _i(aa), _i(al), _d(ae), m, _i(xa), _i(xl), _d(xe),
                         c0, c1, _d(out))
    if rc:
        raise ValueError("angular momentum out of range")
    return out


def _two_index(fn, mol, which):
    if which == "aux":
        n, a, l, e = _basis(mol.aux_atom, mol.aux_l, mol.aux_exp)
        nf = mol.naux
    else:
        n, a, l, e = _basis(mol.ao_atom, mol.ao_l, mol.ao_exp)
        nf = mol.nao
    out = np.zeros((nf, nf))
    xyz = np.ascontiguousarray(mol.coords, np.float64)
    if fn(_d(xyz), n, _i(a), _i(l), _d(e), _d(out)):
        raise ValueError("angular momentum out of range")
    return out


def int2c(mol):
    """Coulomb metric (P|Q)."""
    return _two_index(lib().orc_int2c, mol, "aux")


def overlap(mol):
    """AO overlap matrix."""
    return _two_index(lib().orc_overlap, mol, "ao")


def int4c(mol):
    """(mu nu|la si) over the AO basis, shape (nao,)*4.  Tiny systems only."""
    n, a, l, e = _basis(mol.ao_atom, mol.ao_l, mol.ao_exp)
    nf = mol.nao
    out = np.zeros((nf, nf, nf, nf))
    xyz = np.ascontiguousarray(mol.coords, np.float64)
    if lib().orc_int4c(_d(xyz), n, _i(a), _i(l), _d(e), _d(out)):
        raise ValueError("angular momentum out of range")
    return out


class NotPositiveDefinite(ValueError):
    def __init__(self, pivot):
        super().__init__("metric not positive definite at pivot %d" % pivot)
        self.pivot = pivot


def cholesky(V):
    """Lower-triangular L with V = L L^T (plain column algorithm)."""
    V = np.ascontiguousarray(V, np.float64)
    L = np.zeros_like(V)
    piv = lib().orc_cholesky(V.shape[0], _d(V), _d(L))
    if piv >= 0:
        raise NotPositiveDefinite(int(piv))
    return L


def forward_subst(L, B):
    """X with L X = B (B of shape (n, m)), by plain forward substitution."""
    L = np.ascontiguousarray(L, np.float64)
    X = np.array(B, dtype=np.float64, order="C", copy=True)
    n = L.shape[0]
    m = X.size // n
    lib().orc_forward_subst(n, _d(L), m, _d(X))
    return X


def whitened_3c(mol, U=None):
    """B = L^{-1} U with V = L L^T; returns (B, L) with B shaped (naux, nao, nao)."""
    if U is None:
        U = int3c(mol)
    L = cholesky(int2c(mol))
    B = forward_subst(L, U.reshape(U.shape[0], -1)).reshape(U.shape)
    return B, L


def density(C):
    """Closed-shell density D = 2 C C^T."""
    return 2.0 * C @ C.T


def jk_from_B(B, C=None, D=None):
    """J, K, E_J, E_K from the whitened tensor B (naux, nao, nao)."""
    if (C is None) == (D is None):
        raise ValueError("give exactly one of C and D")
    naux, nao, _ = B.shape
    Bm = B.reshape(naux, nao * nao)
    if C is not None:
        D = density(C)
    c = Bm @ D.ravel()
    J = (c @ Bm).reshape(nao, nao)
    if C is not None:
        X = B @ C                                     # X[P, mu, i]
        K = 2.0 * np.tensordot(X, X, axes=([0, 2], [0, 2]))
    else:
        K = np.zeros((nao, nao))
        for P in range(naux):
            K += B[P] @ D @ B[P]
    EJ = 0.5 * float(np.sum(D * J))
    EK = -0.25 * float(np.sum(D * K))
    return {"J": J, "K": K, "EJ": EJ, "EK": EK, "c": c, "D": D}


def dfjk(mol, C=None, D=None):
    """The full DF-J/K build for a molecule (unscreened)."""
    B, _ = whitened_3c(mol)
    return jk_from_B(B, C=C, D=D)


def uks_from_B(B, Ca, Cb):
    """Open-shell (unrestricted) J/K from B: per spin D_s = C_s C_s^T and
    K_s = sum_P B_P D_s B_P; J from D = D_a + D_b; E_J = 1/2 Tr(D J),
    E_K = -1/2 (Tr D_a K_a + Tr D_b K_b).  The paper lists unrestricted SCF
    among the GPU-optimised methods (Section "Accelerated Functionalities",
    table of functionalities); the formulas are the standard spin-unrestricted
    Coulomb and exchange terms."""
    naux, nao, _ = B.shape
    Bm = B.reshape(naux, nao * nao)
    Ds = [C @ C.T for C in (Ca, Cb)]
    D = Ds[0] + Ds[1]
    c = Bm @ D.ravel()
    J = (c @ Bm).reshape(nao, nao)
    Ks = []
    for Dsp in Ds:
        K = np.zeros((nao, nao))
        for P in range(naux):
            K += B[P] @ Dsp @ B[P]
        Ks.append(K)
    EJ = 0.5 * float(np.sum(D * J))
    EK = -0.5 * float(np.sum(Ds[0] * Ks[0]) + np.sum(Ds[1] * Ks[1]))
    return {"J": J, "Ka": Ks[0], "Kb": Ks[1], "EJ": EJ, "EK": EK}


def dfjk_uks(mol, Ca, Cb):
    """Unrestricted DF-J/K for a molecule (unscreened)."""
    B, _ = whitened_3c(mol)
    return uks_from_B(B, Ca, Cb)


def exact_jk_blocks(mol, D, shell_pairs):
    """Exact (unfitted, unscreened) J and K blocks for the AO shell pairs
    (a, c) listed, from the four-centre definitions
    J_{mu nu} = sum_{la si} (mu nu|la si) D_{la si} and
    K_{mu nu} = sum_{la si} (mu la|nu si) D_{la si}, mu in shell a, nu in c.
    Returns two lists of (2l_a+1, 2l_c+1) arrays.  The cost per block is one
    pass over every shell pair of the basis, so this reaches single blocks of
    molecules far too large for the dense tensor."""
    n, a, l, e = _basis(mol.ao_atom, mol.ao_l, mol.ao_exp)
    pairs = np.asarray(shell_pairs, dtype=np.int32).reshape(-1, 2)
    ra = np.ascontiguousarray(pairs[:, 0]); rc = np.ascontiguousarray(pairs[:, 1])
    sizes = (2 * mol.ao_l[ra] + 1) * (2 * mol.ao_l[rc] + 1)
    boff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    J = np.zeros(int(boff[-1])); K = np.zeros(int(boff[-1]))
    xyz = np.ascontiguousarray(mol.coords, np.float64)
    Dc = np.ascontiguousarray(D, np.float64)
    rc_ = lib().orc_jk_blocks(_d(xyz), n, _i(a), _i(l), _d(e), _d(Dc), len(pairs), _i(ra), _i(rc),
                              boff[:-1].ctypes.data_as(ctypes.POINTER(ctypes.c_long)), _d(J), _d(K))
    if rc_:
        raise ValueError("angular momentum or shell index out of range")
    shp = [(2 * int(mol.ao_l[x]) + 1, 2 * int(mol.ao_l[y]) + 1) for x, y in pairs]
    Js = [J[boff[k]:boff[k + 1]].reshape(shp[k]) for k in range(len(pairs))]
    Ks = [K[boff[k]:boff[k + 1]].reshape(shp[k]) for k in range(len(pairs))]
    return Js, Ks


def exact_jk(mol, D):
    """Exact (non-fitted) J and K from four-centre integrals (tiny systems)."""
    eri = int4c(mol)
    J = np.einsum("mnls,ls->mn", eri, D)
    K = np.einsum("mlns,ls->mn", eri, D)
    return J, K, 0.5 * float(np.sum(D * J)), -0.25 * float(np.sum(D * K))


def dfjk_streamed(mol, Cs, rows, shell_step=16):
    """Fitted J/K energies and sampled rows for molecules too large for the
    dense path, from the same textbook definitions evaluated one slice of
    auxiliary shells at a time (unscreened):

        u_Q = sum_{mu nu} (mu nu|Q) D_{mu nu},  c = L^{-1} u,  E_J = 1/2 c.c
        J_{mu nu} = sum_Q (mu nu|Q) w_Q,        w = L^{-T} c
        T_{Q,mu i} = sum_nu (mu nu|Q) C_{nu i}, X = L^{-1} T
        K = 2 sum_{P,i} X_{P,mu i} X_{P,nu i},  E_K = -1/4 Tr(D K)

    with D = 2 C C^T and V = (P|Q) = L L^T.  This is J = sum_P B_P c_P and
    the half-transform route of K with B = L^{-1} U, rearranged so that
    neither U nor B is held whole (the (mu nu|Q) slices are recomputed for
    the J pass).  Cs is a list of (nao, nocc) orbital matrices; returns one
    dict per entry with E_J, E_K and the K and J rows listed in `rows`."""
    import scipy.linalg

    nao, naux = mol.nao, mol.naux
    Ds = [density(C) for C in Cs]
    L = cholesky(int2c(mol))
    nsh = len(mol.aux_l)
    u = [np.zeros(naux) for _ in Cs]
    T = [np.zeros((naux, nao, C.shape[1])) for C in Cs]
    p = 0
    for c0 in range(0, nsh, shell_step):
        U = int3c(mol, c0, min(nsh, c0 + shell_step))
        m = U.shape[0]
        for k, C in enumerate(Cs):
            u[k][p:p + m] = U.reshape(m, -1) @ Ds[k].ravel()
            T[k][p:p + m] = U @ C
        p += m
    rows = np.asarray(rows, dtype=np.int64)
    out = []
    for k, C in enumerate(Cs):
        c = forward_subst(L, u[k][:, None])[:, 0]
        X = forward_subst(L, T[k].reshape(naux, -1)).reshape(naux, nao, C.shape[1])
        T[k] = None
        A = np.ascontiguousarray(X.transpose(1, 0, 2)).reshape(nao, -1)
        del X
        K = 2.0 * (A @ A.T)
        del A
        out.append({"E_J": 0.5 * float(c @ c), "E_K": -0.25 * float(np.sum(Ds[k] * K)),
                    "K_rows": K[rows].copy(), "c": c,
                    "w": scipy.linalg.solve_triangular(L, c, trans="T", lower=True)})
    Jr = [np.zeros((len(rows), nao)) for _ in Cs]
    p = 0
    for c0 in range(0, nsh, shell_step):
        U = int3c(mol, c0, min(nsh, c0 + shell_step))
        m = U.shape[0]
        Ur = U[:, rows, :]
        for k in range(len(Cs)):
            Jr[k] += np.tensordot(out[k]["w"][p:p + m], Ur, axes=(0, 0))
        p += m
    for k in range(len(Cs)):
        out[k]["J_rows"] = Jr[k]
    return out
