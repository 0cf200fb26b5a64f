"""Pins for the CPU oracle, checked against things other than itself:
closed forms, a library routine, brute-force quadrature, exactness cases and
invariants of Coulomb-metric density fitting.  All CPU-only."""
import math
import os

import numpy as np
import pytest
import scipy.linalg
import scipy.special

import oracle
import workload as W
from tests import brute


def _mol(ao, aux, coords, charges=None):
    """Molecule from explicit shell lists [(atom, l, exp), ...]."""
    coords = np.asarray(coords, float)
    if charges is None:
        charges = np.zeros(len(coords), int)
    ao = np.array(ao, dtype=object)
    aux = np.array(aux, dtype=object)
    return W.Molecule(charges=np.asarray(charges), coords=coords,
                      ao_atom=ao[:, 0].astype(np.int32), ao_l=ao[:, 1].astype(np.int32),
                      ao_exp=ao[:, 2].astype(float),
                      aux_atom=aux[:, 0].astype(np.int32), aux_l=aux[:, 1].astype(np.int32),
                      aux_exp=aux[:, 2].astype(float))


@pytest.fixture(scope="module")
def water():
    z, x = W.water_monomer()
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C = W.occupied_orbitals(S, 5, 0)
    return mol, S, C


# --------------------------------------------------------------------------
# Boys function

def _boys_mp(m, T):
    import mpmath
    mpmath.mp.dps = 50
    if T == 0:
        return 1.0 / (2 * m + 1)
    T = mpmath.mpf(T)
    return float(mpmath.gammainc(m + mpmath.mpf(1) / 2, 0, T) / (2 * T ** (m + mpmath.mpf(1) / 2)))


def test_boys_against_mpmath():
    Ts = list(np.linspace(0.0, 40.0, 81)) + list(np.logspace(-10, np.log10(200.0), 40)) + [29.999, 30.001]
    worst = 0.0
    for T in Ts:
        F = oracle.boys(8, T)
        for m in range(9):
            ref = _boys_mp(m, T)
            worst = max(worst, abs(F[m] - ref) / ref)
    assert worst <= 1e-14, worst


def test_boys_special_values():
    F = oracle.boys(12, 0.0)
    assert np.allclose(F, [1.0 / (2 * m + 1) for m in range(13)], rtol=0, atol=1e-16)
    for T in (1e-3, 0.7, 3.0, 12.0, 31.0, 90.0):
        F = oracle.boys(8, T)
        assert abs(F[0] - 0.5 * math.sqrt(math.pi / T) * math.erf(math.sqrt(T))) <= 1e-15 * F[0]
        for m in range(9):                       # Kummer form
            ref = scipy.special.hyp1f1(m + 0.5, m + 1.5, -T) / (2 * m + 1)
            assert abs(F[m] - ref) <= 1e-12 * ref
        for m in range(8):                       # downward-recursion identity
            assert abs((2 * m + 1) * F[m] - (2 * T * F[m + 1] + math.exp(-T))) <= 1e-14 * (2 * m + 1) * F[m]


def test_boys_large_T_asymptote():
    for T in (80.0, 150.0, 400.0):
        F = oracle.boys(8, T)
        for m in range(9):
            dfm = np.prod(np.arange(2 * m - 1, 0, -2)) if m > 0 else 1.0
            asym = dfm / 2 ** (m + 1) * math.sqrt(math.pi / T ** (2 * m + 1))
            assert abs(F[m] - asym) <= 1e-14 * asym


# --------------------------------------------------------------------------
# Normalisation, overlap and the spherical convention

def test_overlap_unit_diagonal_and_one_centre_identity():
    mol = _mol([(0, l, e) for l in range(4) for e in (0.3, 2.0)], [(0, 0, 1.0)], [[0.1, 0.2, 0.3]])
    S = oracle.overlap(mol)
    off = np.concatenate([[0], np.cumsum(2 * mol.ao_l + 1)])
    assert np.abs(np.diag(S) - 1).max() <= 1e-14
    for k in range(len(mol.ao_l)):
        blk = S[off[k]:off[k + 1], off[k]:off[k + 1]]
        assert np.abs(blk - np.eye(len(blk))).max() <= 1e-14


def test_norm_against_numeric_radial_integral():
    for l in range(4):
        for a in (0.05, 1.0, 700.0):
            # Racah-normalised angular part integrates to 4 pi / (2l+1)
            radial = scipy.special.gamma(l + 1.5) / (2 * (2 * a) ** (l + 1.5))
            N = oracle.norm(l, a)
            assert abs(N * N * radial * 4 * math.pi / (2 * l + 1) - 1.0) <= 1e-13


def test_overlap_matches_generator_quadrature(water):
    mol, S_quad, C = water
    S = oracle.overlap(mol)
    assert np.abs(S - S_quad).max() <= 1e-13
    # shells up to f on several centres, against the quadrature too
    mol2 = _mol([(0, 3, 0.9), (1, 2, 0.5), (2, 1, 1.7), (0, 0, 3.0), (1, 3, 0.4)],
                [(0, 0, 1.0)], [[0, 0, 0], [0.8, -0.4, 0.3], [-0.5, 0.6, 1.1]])
    assert np.abs(oracle.overlap(mol2) - W.overlap_by_quadrature(mol2)).max() <= 1e-13


def test_density_trace_is_electron_count(water):
    mol, S_quad, C = water
    D = oracle.density(C)
    assert abs(np.sum(D * oracle.overlap(mol)) - mol.nelec) <= 1e-12


# --------------------------------------------------------------------------
# Integrals: closed forms and brute force

def test_ss_s_and_s_s_and_ssss_closed_forms():
    A, B, C = np.array([0.0, 0, 0]), np.array([0.9, -0.3, 0.4]), np.array([-0.6, 1.2, 0.2])
    a, b, g = 1.7, 0.45, 0.8
    mol = _mol([(0, 0, a), (1, 0, b)], [(2, 0, g), (0, 0, 2.3)], [A, B, C])
    U = oracle.int3c(mol)
    n = lambda e: (2 * e / math.pi) ** 0.75
    p = a + b
    P = (a * A + b * B) / p
    al = p * g / (p + g)
    ref = (n(a) * n(b) * n(g) * 2 * math.pi ** 2.5 / (p * g * math.sqrt(p + g))
           * math.exp(-a * b / p * np.sum((A - B) ** 2)) * brute.boys0(al * np.sum((P - C) ** 2)))
    assert abs(U[0, 0, 1] - ref) <= 1e-14 * ref
    assert U[0, 0, 1] == U[0, 1, 0]
    V = oracle.int2c(mol)
    g2 = 2.3
    ref2 = n(g) * n(g2) * 2 * math.pi ** 2.5 / (g * g2 * math.sqrt(g + g2)) * brute.boys0(
        g * g2 / (g + g2) * np.sum((C - A) ** 2))
    assert abs(V[0, 1] - ref2) <= 1e-14 * ref2
    # self-repulsion of one normalised s: (aa|aa) = 2 sqrt(a/pi)
    eri = oracle.int4c(_mol([(0, 0, a)], [(0, 0, 1.0)], [A]))
    assert abs(eri[0, 0, 0, 0] - 2 * math.sqrt(a / math.pi)) <= 1e-14
    # a generic (ss|ss) against the closed form
    eri = oracle.int4c(mol)
    ref4 = brute.ssss(a, A, b, B, b, B, a, A)
    assert abs(eri[0, 1, 1, 0] - ref4) <= 1e-14 * ref4


@pytest.mark.parametrize("la,lb,lc", [(1, 0, 0), (0, 0, 1), (1, 1, 2), (2, 0, 3), (2, 1, 1), (2, 2, 3), (0, 2, 2)])
def test_int3c_against_t_quadrature(la, lb, lc):
    A, B, C = [0.2, -0.1, 0.3], [1.1, 0.6, -0.5], [-0.4, 0.9, 0.7]
    a, b, g = 1.4, 0.55, 0.95
    mol = _mol([(0, la, a), (1, lb, b)], [(2, lc, g)], [A, B, C])
    U = oracle.int3c(mol)
    na, nb = 2 * la + 1, 2 * lb + 1
    got = U[:, 0:na, na:na + nb].transpose(1, 2, 0)
    ref = brute.coulomb3c_block(la, a, A, lb, b, B, lc, g, C)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_int3c_same_centre_against_t_quadrature():
    A = [0.3, 0.2, -0.4]
    mol = _mol([(0, 2, 0.8), (0, 1, 2.2)], [(0, 3, 1.5)], [A])
    U = oracle.int3c(mol)
    got = U[:, 0:5, 5:8].transpose(1, 2, 0)
    ref = brute.coulomb3c_block(2, 0.8, A, 1, 2.2, A, 3, 1.5, A)
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_int3c_shell_order_reversal():
    """Reversing the AO shell list swaps the roles of the two E recursions."""
    z, x = W.water_monomer()
    mol = W.make_molecule(z, x)
    U = oracle.int3c(mol)
    rev = _mol(list(zip(mol.ao_atom[::-1], mol.ao_l[::-1], mol.ao_exp[::-1])),
               list(zip(mol.aux_atom, mol.aux_l, mol.aux_exp)), mol.coords)
    Ur = oracle.int3c(rev)
    off = np.concatenate([[0], np.cumsum(2 * mol.ao_l + 1)])
    perm = np.concatenate([np.arange(off[k], off[k + 1]) for k in range(len(mol.ao_l))[::-1]])
    assert np.abs(Ur - U[:, perm][:, :, perm]).max() <= 1e-13 * np.abs(U).max()


@pytest.mark.parametrize("la,lb,lc,ld", [(1, 0, 0, 0), (0, 0, 1, 1), (1, 1, 1, 0), (2, 0, 1, 1),
                                         (2, 1, 2, 0), (2, 2, 1, 1), (1, 2, 2, 2)])
def test_int4c_against_t_quadrature(la, lb, lc, ld):
    """Four-centre blocks on four distinct centres against the quadrature,
    which shares neither the Boys function nor the Hermite recursions."""
    cen = [[0.2, -0.1, 0.3], [1.1, 0.6, -0.5], [-0.4, 0.9, 0.7], [0.5, -0.6, -0.2]]
    ex = [1.4, 0.55, 0.95, 2.1]
    ls = [la, lb, lc, ld]
    mol = _mol([(k, ls[k], ex[k]) for k in range(4)], [(0, 0, 1.0)], cen)
    eri = oracle.int4c(mol)
    o = np.concatenate([[0], np.cumsum([2 * l + 1 for l in ls])])
    got = eri[o[0]:o[1], o[1]:o[2], o[2]:o[3], o[3]:o[4]]
    ref = brute.coulomb4c_block(la, ex[0], cen[0], lb, ex[1], cen[1], lc, ex[2], cen[2], ld, ex[3], cen[3])
    assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()


def test_int4c_permutation_symmetry(water):
    mol, _, _ = water
    eri = oracle.int4c(mol)
    for perm in [(1, 0, 2, 3), (0, 1, 3, 2), (2, 3, 0, 1)]:
        assert np.abs(eri - eri.transpose(perm)).max() <= 1e-13 * np.abs(eri).max()


def test_exact_jk_blocks_equal_dense_definition(water):
    """The block routine (one pass over every shell pair per block) against
    the dense tensor contracted by einsum, on every block of the monomer."""
    mol, _, C = water
    D = oracle.density(C)
    J, K, _, _ = oracle.exact_jk(mol, D)
    off = np.concatenate([[0], np.cumsum(2 * mol.ao_l + 1)])
    ns = len(mol.ao_l)
    pairs = [(a, c) for a in range(ns) for c in range(ns)]
    Js, Ks = oracle.exact_jk_blocks(mol, D, pairs)
    for (a, c), jb, kb in zip(pairs, Js, Ks):
        assert np.abs(jb - J[off[a]:off[a + 1], off[c]:off[c + 1]]).max() <= 1e-13 * np.abs(J).max()
        assert np.abs(kb - K[off[a]:off[a + 1], off[c]:off[c + 1]]).max() <= 1e-13 * np.abs(K).max()


def test_exact_jk_structure(water):
    """J and K symmetric, K positive semidefinite for D = 2 C C^T, E_J > 0,
    E_K < 0, and both linear in D."""
    mol, _, C = water
    D = oracle.density(C)
    J, K, EJ, EK = oracle.exact_jk(mol, D)
    assert np.abs(J - J.T).max() <= 1e-13 * np.abs(J).max()
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    assert np.linalg.eigvalsh(0.5 * (K + K.T)).min() >= -1e-12 * np.abs(K).max()
    assert EJ > 0 and EK < 0
    rng = np.random.default_rng(5)
    M = rng.standard_normal(D.shape)
    D2 = M + M.T
    J2, K2, _, _ = oracle.exact_jk(mol, D2)
    J3, K3, _, _ = oracle.exact_jk(mol, 0.5 * D - 2.0 * D2)
    assert np.abs(J3 - (0.5 * J - 2.0 * J2)).max() <= 1e-12 * np.abs(J3).max()
    assert np.abs(K3 - (0.5 * K - 2.0 * K2)).max() <= 1e-12 * np.abs(K3).max()


def test_int2c_equals_int3c_with_flat_partner():
    """(P|Q) is (P s_eps|Q) / N_0(eps) for a vanishing-exponent s partner."""
    coords = [[0, 0, 0], [0.7, -0.2, 0.5], [-0.3, 0.8, 0.1]]
    aux_shells = [(0, 0, 1.2), (1, 1, 0.7), (2, 2, 1.9), (0, 3, 0.8)]
    eps = 1e-10
    for sh in aux_shells:
        mol3 = _mol([sh, (0, 0, eps)], aux_shells, coords)
        U = oracle.int3c(mol3)
        n1 = 2 * sh[1] + 1
        got = U[:, 0:n1, n1] / oracle.norm(0, eps)
        V = oracle.int2c(_mol([(0, 0, 1.0)], aux_shells, coords))
        k = aux_shells.index(sh)
        off = np.concatenate([[0], np.cumsum([2 * s[1] + 1 for s in aux_shells])])
        ref = V[:, off[k]:off[k + 1]]
        assert np.abs(got - ref).max() <= 1e-8 * np.abs(ref).max()


def test_schwarz_inequality_holds(water):
    mol, _, _ = water
    U = oracle.int3c(mol)
    eri = oracle.int4c(mol)
    V = oracle.int2c(mol)
    n = mol.nao
    diag = np.sqrt(np.abs(eri.reshape(n * n, n * n).diagonal())).reshape(n, n)
    bound = diag[None, :, :] * np.sqrt(np.diag(V))[:, None, None]
    assert np.all(np.abs(U) <= bound * (1 + 1e-12) + 1e-300)


# --------------------------------------------------------------------------
# Linear algebra

def test_cholesky_and_forward_substitution_against_lapack(water):
    mol, _, _ = water
    V = oracle.int2c(mol)
    L = oracle.cholesky(V)
    assert np.allclose(np.triu(L, 1), 0.0)
    assert np.abs(L @ L.T - V).max() <= 1e-14 * np.abs(V).max()
    assert np.abs(L - np.linalg.cholesky(V)).max() <= 1e-12 * np.abs(L).max()
    rng = np.random.default_rng(3)
    Bm = rng.standard_normal((V.shape[0], 700))
    X = oracle.forward_subst(L, Bm)
    ref = scipy.linalg.solve_triangular(L, Bm, lower=True)
    assert np.abs(X - ref).max() <= 1e-11 * np.abs(ref).max()


def test_cholesky_reports_nonpositive_pivot():
    A = np.array([[4.0, 2.0, 0.0], [2.0, 1.0, 1.0], [0.0, 1.0, 3.0]])   # pivot 1 is 0
    with pytest.raises(oracle.NotPositiveDefinite) as ei:
        oracle.cholesky(A)
    assert ei.value.pivot == 1
    with pytest.raises(oracle.NotPositiveDefinite) as ei:
        oracle.cholesky(np.diag([1.0, 2.0, -1.0]))
    assert ei.value.pivot == 2


# --------------------------------------------------------------------------
# DF-J/K: exactness, bounds and invariants

def test_df_exact_one_centre():
    a = 1.3
    mol = _mol([(0, 0, a)], [(0, 0, 2 * a)], [[0.0, 0.0, 0.0]])
    r = oracle.dfjk(mol, D=np.array([[2.0]]))
    assert abs(r["EJ"] - 4 * math.sqrt(a / math.pi)) <= 1e-14
    assert abs(r["EK"] + 2 * math.sqrt(a / math.pi)) <= 1e-14


def test_df_exact_two_centre():
    """Aux {2a@A, 2b@B, (a+b)@P} spans every AO product: DF J/K equal the exact 4c J/K."""
    A, B = np.array([0.0, 0.0, 0.0]), np.array([0.4, -0.3, 0.5])
    a, b = 0.9, 1.6
    P = (a * A + b * B) / (a + b)
    mol = _mol([(0, 0, a), (1, 0, b)], [(0, 0, 2 * a), (1, 0, 2 * b), (2, 0, a + b)], [A, B, P])
    rng = np.random.default_rng(0)
    M = rng.standard_normal((2, 2))
    D = M + M.T
    r = oracle.dfjk(mol, D=D)
    cen, ex = [A, B], [a, b]
    eri = np.zeros((2, 2, 2, 2))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    eri[i, j, k, l] = brute.ssss(ex[i], cen[i], ex[j], cen[j], ex[k], cen[k], ex[l], cen[l])
    J = np.einsum("ijkl,kl->ij", eri, D)
    K = np.einsum("ikjl,kl->ij", eri, D)
    assert np.abs(r["J"] - J).max() <= 1e-12 * np.abs(J).max()
    assert np.abs(r["K"] - K).max() <= 1e-12 * np.abs(K).max()


def test_df_variational_bounds(water):
    mol, _, C = water
    D = oracle.density(C)
    r = oracle.dfjk(mol, C=C)
    _, _, EJ, EK = oracle.exact_jk(mol, D)
    assert r["EJ"] <= EJ + 1e-12
    assert abs(r["EK"]) <= abs(EK) + 1e-12


def test_k_routes_agree_with_literal_four_index_sum(water):
    mol, _, C = water
    B, _ = oracle.whitened_3c(mol)
    D = oracle.density(C)
    viaC = oracle.jk_from_B(B, C=C)
    viaD = oracle.jk_from_B(B, D=D)
    eri_df = np.einsum("Pml,Pns->mlns", B, B)        # (ml|ns)_DF
    K = np.einsum("mlns,ls->mn", eri_df, D)
    J = np.einsum("mnls,ls->mn", eri_df, D)
    s = np.abs(K).max()
    assert np.abs(viaC["K"] - K).max() <= 1e-13 * s
    assert np.abs(viaD["K"] - K).max() <= 1e-13 * s
    assert np.abs(viaC["J"] - J).max() <= 1e-13 * np.abs(J).max()


def test_jk_structure_and_energy_identities(water):
    mol, _, C = water
    B, _ = oracle.whitened_3c(mol)
    r = oracle.jk_from_B(B, C=C)
    J, K = r["J"], r["K"]
    assert np.abs(J - J.T).max() <= 1e-13 * np.abs(J).max()
    assert np.abs(K - K.T).max() <= 1e-13 * np.abs(K).max()
    assert np.linalg.eigvalsh(0.5 * (K + K.T)).min() >= -1e-12 * np.abs(K).max()
    assert abs(r["EJ"] - 0.5 * np.sum(r["c"] ** 2)) <= 1e-12 * abs(r["EJ"])
    Bij = np.einsum("mi,Pmn,nj->Pij", C, B, C)
    assert abs(r["EK"] + np.sum(Bij ** 2)) <= 1e-12 * abs(r["EK"])
    # linearity in D
    rng = np.random.default_rng(5)
    M = rng.standard_normal(J.shape)
    D1, D2 = M + M.T, r["D"]
    ra, rb = oracle.jk_from_B(B, D=D1), oracle.jk_from_B(B, D=D2)
    rs = oracle.jk_from_B(B, D=0.3 * D1 + 1.7 * D2)
    assert np.abs(rs["J"] - (0.3 * ra["J"] + 1.7 * rb["J"])).max() <= 1e-12 * np.abs(rs["J"]).max()
    assert np.abs(rs["K"] - (0.3 * ra["K"] + 1.7 * rb["K"])).max() <= 1e-12 * np.abs(rs["K"]).max()


def test_aux_permutation_invariance(water):
    mol, _, C = water
    r = oracle.dfjk(mol, C=C)
    perm = np.random.default_rng(11).permutation(len(mol.aux_l))
    mol2 = _mol(list(zip(mol.ao_atom, mol.ao_l, mol.ao_exp)),
                list(zip(mol.aux_atom[perm], mol.aux_l[perm], mol.aux_exp[perm])), mol.coords)
    r2 = oracle.dfjk(mol2, C=C)
    assert np.abs(r2["J"] - r["J"]).max() <= 1e-11 * np.abs(r["J"]).max()
    assert np.abs(r2["K"] - r["K"]).max() <= 1e-11 * np.abs(r["K"]).max()


def test_translation_invariance(water):
    mol, _, C = water
    r = oracle.dfjk(mol, C=C)
    r2 = oracle.dfjk(W.shift_molecule(mol, [3.1, -2.2, 0.7]), C=C)
    for k in ("J", "K"):
        assert np.abs(r2[k] - r[k]).max() <= 1e-10 * np.abs(r[k]).max()


def test_atom_relabelling_permutes_jk():
    z, x = W.water_cluster(2, 6.0, 21)
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C = W.occupied_orbitals(S, 10, 2)
    r = oracle.dfjk(mol, C=C)
    order = [3, 4, 5, 0, 1, 2]                      # swap the two waters
    mol2 = W.make_molecule(z[order], x[order])
    # AO functions of mol2 in terms of mol: the second water's block first
    half = mol.nao // 2
    perm = np.concatenate([np.arange(half, mol.nao), np.arange(half)])
    r2 = oracle.dfjk(mol2, C=C[perm])
    assert np.abs(r2["J"] - r["J"][np.ix_(perm, perm)]).max() <= 1e-10 * np.abs(r["J"]).max()
    assert np.abs(r2["K"] - r["K"][np.ix_(perm, perm)]).max() <= 1e-10 * np.abs(r["K"]).max()


def test_far_dimer_exchange_approaches_additivity():
    """E_K(AB) - E_K(A) - E_K(B) for block-diagonal orbitals decays with R
    (a power law from the long-range tail of the fitted pair densities)."""
    z, x = W.water_monomer()
    mon = W.make_molecule(z, x)
    S1 = W.overlap_by_quadrature(mon)
    C1 = W.occupied_orbitals(S1, 5, 0)
    EK1 = oracle.dfjk(mon, C=C1)["EK"]
    diffs = []
    for R in (20.0, 40.0, 80.0):
        xyz = np.vstack([x, x + np.array([R, 0.0, 0.0])])
        dim = W.make_molecule(np.concatenate([z, z]), xyz)
        C = np.zeros((2 * mon.nao, 10))
        C[:mon.nao, :5] = C1
        C[mon.nao:, 5:] = C1
        diffs.append(abs(oracle.dfjk(dim, C=C)["EK"] - 2 * EK1))
    assert diffs[0] > diffs[1] > diffs[2]
    assert diffs[2] < 1e-3 * abs(EK1)


# --------------------------------------------------------------------------
# Open shell (unrestricted)

def test_uks_closed_shell_reduction(water):
    """C_a = C_b = C gives the closed-shell result: K_a = K_b = K / 2, same J and energies."""
    mol, _, C = water
    B, _ = oracle.whitened_3c(mol)
    r = oracle.jk_from_B(B, C=C)
    u = oracle.uks_from_B(B, C, C)
    s = np.abs(r["K"]).max()
    assert np.abs(u["J"] - r["J"]).max() <= 1e-13 * np.abs(r["J"]).max()
    assert np.abs(u["Ka"] - 0.5 * r["K"]).max() <= 1e-13 * s
    assert np.abs(u["Kb"] - 0.5 * r["K"]).max() <= 1e-13 * s
    assert abs(u["EJ"] - r["EJ"]) <= 1e-13 * abs(r["EJ"])
    assert abs(u["EK"] - r["EK"]) <= 1e-13 * abs(r["EK"])


def test_uks_one_electron_has_no_self_interaction(water):
    """One electron (one alpha orbital, no beta): E_J + E_K = 0, as Coulomb and
    exchange of a single orbital density cancel term by term in P."""
    mol, _, C = water
    B, _ = oracle.whitened_3c(mol)
    u = oracle.uks_from_B(B, C[:, :1], C[:, :0])
    assert u["EJ"] > 0
    assert abs(u["EJ"] + u["EK"]) <= 1e-13 * u["EJ"]
    assert np.all(u["Kb"] == 0.0)


def test_uks_exact_two_centre_against_brute_force():
    """With an aux set spanning every AO product, each spin's K equals the exact
    four-centre exchange of its own density (brute-force (ss|ss))."""
    A, Bc = np.array([0.0, 0.0, 0.0]), np.array([0.4, -0.3, 0.5])
    a, b = 0.9, 1.6
    P = (a * A + b * Bc) / (a + b)
    mol = _mol([(0, 0, a), (1, 0, b)], [(0, 0, 2 * a), (1, 0, 2 * b), (2, 0, a + b)], [A, Bc, P])
    rng = np.random.default_rng(5)
    Ca, Cb = rng.standard_normal((2, 2)), rng.standard_normal((2, 1))
    u = oracle.dfjk_uks(mol, Ca, Cb)
    cen, ex = [A, Bc], [a, b]
    eri = np.zeros((2, 2, 2, 2))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    eri[i, j, k, l] = brute.ssss(ex[i], cen[i], ex[j], cen[j], ex[k], cen[k], ex[l], cen[l])
    Da, Db = Ca @ Ca.T, Cb @ Cb.T
    J = np.einsum("ijkl,kl->ij", eri, Da + Db)
    Ka, Kb = np.einsum("ikjl,kl->ij", eri, Da), np.einsum("ikjl,kl->ij", eri, Db)
    assert np.abs(u["J"] - J).max() <= 1e-12 * np.abs(J).max()
    assert np.abs(u["Ka"] - Ka).max() <= 1e-12 * np.abs(Ka).max()
    assert np.abs(u["Kb"] - Kb).max() <= 1e-12 * np.abs(Kb).max()
    EK = -0.5 * (np.sum(Da * Ka) + np.sum(Db * Kb))
    assert abs(u["EK"] - EK) <= 1e-12 * abs(EK)


def test_streamed_route_equals_dense_definition():
    """The slice-by-slice evaluation used for large clusters (oracle.dfjk_streamed)
    gives the dense path's E_J, E_K and J/K rows (3 waters, ragged last slice)."""
    import workload as W
    mol, S, C = W.build_case(3, geom_seed=103)
    C2 = W.perturbed_orbitals(C, S, 1)
    rows = [0, 5, 17, 44, 89]
    res = oracle.dfjk_streamed(mol, [C, C2], rows, shell_step=7)
    for Ck, r in zip([C, C2], res):
        ref = oracle.dfjk(mol, C=Ck)
        assert abs(r["E_J"] - ref["EJ"]) <= 1e-13 * abs(ref["EJ"])
        assert abs(r["E_K"] - ref["EK"]) <= 1e-13 * abs(ref["EK"])
        assert np.abs(r["K_rows"] - ref["K"][rows]).max() <= 1e-13 * np.abs(ref["K"]).max()
        assert np.abs(r["J_rows"] - ref["J"][rows]).max() <= 1e-13 * np.abs(ref["J"]).max()


def test_golden_water32_fixture_is_consistent():
    """The stored 32-water oracle values obey the structure every fitted K has:
    K rows are the rows of a symmetric matrix (K[r_a][r_b] = K[r_b][r_a]),
    E_J > 0 > E_K, and builds 0 and 9 differ by a small orbital step."""
    import json
    path = os.path.join(os.path.dirname(__file__), "golden", "water32.json")
    if not os.path.exists(path):
        pytest.skip("water32.json not generated")
    g = json.load(open(path))
    rows = g["rows"]
    for b in g["builds"].values():
        K = np.asarray(b["K_rows"])
        assert K.shape == (len(rows), g["nao"])
        sub = K[:, rows]
        assert np.abs(sub - sub.T).max() <= 1e-12 * np.abs(K).max()
        J = np.asarray(b["J_rows"])
        subj = J[:, rows]
        assert np.abs(subj - subj.T).max() <= 1e-12 * np.abs(J).max()
        assert b["E_J"] > 0 > b["E_K"]
        # diagonal of K for D = 2 C C^T is >= 0 (K is positive semidefinite)
        assert np.all(np.diag(sub) >= 0)
    e0, e9 = g["builds"]["0"], g["builds"]["9"]
    assert abs(e0["E_K"] - e9["E_K"]) < 0.05 * abs(e0["E_K"])


# ---------------------------------------------------------------------------
# Mixed-precision formats (oracle.mixed)

def test_bf16_rounding_matches_torch():
    """The bf16 rounding of oracle.mixed equals torch's float32 -> bfloat16
    conversion (round to nearest even), ties and subnormals included."""
    torch = pytest.importorskip("torch")
    from oracle import mixed as M
    rng = np.random.default_rng(5)
    x = np.concatenate([rng.standard_normal(20000) * 10.0 ** rng.integers(-30, 30, 20000),
                        np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -1.0 - 2.0 ** -8, 1e-40, -3e-39])])
    x32 = x.astype(np.float32)
    ref = torch.from_numpy(x32).to(torch.bfloat16).to(torch.float64).numpy()
    assert np.array_equal(M._bf16(x32), ref)
    hi, lo = M.split_bf16(x)
    xs = x32.astype(np.float64)
    normal = np.abs(xs) > 1e-30          # lo stays a normal number
    assert np.all(np.abs(hi + lo - xs)[normal] <= 2.0 ** -17 * np.abs(xs)[normal])


def test_int8_slices_digits_and_reconstruction():
    from oracle import mixed as M
    rng = np.random.default_rng(6)
    X = rng.standard_normal((7, 1024)) * 10.0 ** rng.uniform(-12, 3, (7, 1024))
    X[3, 256:512] = 0.0                                  # an all-zero block
    X[4, 0] = 127.0 / 128.0 * 4.0                        # block max on the scale boundary
    a, e = M.int8_slices(X, block=256, nslices=5)
    assert np.abs(a[0]).max() <= 127 and all(np.abs(s).max() <= 64 for s in a[1:])
    m = np.abs(X.reshape(7, 4, 256)).max(axis=2)
    nz = m > 0
    # e is the least integer with 2^e > max|x| 128/127
    assert np.all(np.ldexp(1.0, e[nz]) > m[nz] * 128 / 127)
    assert np.all(np.ldexp(1.0, e[nz] - 1) <= m[nz] * 128 / 127)
    rec = sum(np.ldexp(s, -7 * (k + 1)) for k, s in enumerate(a)).reshape(7, 4, 256)
    rec = rec * np.ldexp(1.0, e)[:, :, None]
    scale = np.ldexp(1.0, e)[:, :, None] * np.ones((1, 1, 256))
    assert np.all(np.abs(rec - X.reshape(7, 4, 256)) <= 2.0 ** -36 * scale)
    assert np.all(a[0][3, 256:512] == 0)


def test_int8_product_truncation_bound_and_limit():
    """Kept orders i + j <= 4 stay within 2^-33 of the scale envelope of the
    exact product; keeping every product of eight slices approaches it to
    FP64 level (the slicing itself is exact)."""
    from oracle import mixed as M
    rng = np.random.default_rng(7)
    A = rng.standard_normal((20, 512)) * 10.0 ** rng.uniform(-6, 1, (20, 512))
    B = rng.standard_normal((12, 512)) * 10.0 ** rng.uniform(-6, 1, (12, 512))
    exact = A @ B.T
    S = M.int8_scale_envelope(A, B)
    P = M.int8_product(A, B)
    assert np.all(np.abs(P - exact) <= 2.0 ** -33 * S)
    assert np.abs(P - exact).max() > 0
    P8 = M.int8_product(A, B, nslices=8, keep=lambda i, j: True)
    assert np.all(np.abs(P8 - exact) <= 2.0 ** -48 * S + 1e-15 * np.abs(A) @ np.abs(B).T)


def _x_rows_water3():
    """X of 3 waters (the mixed GPU test's case) as contraction rows, aux
    functions in the library's internal order (shells sorted by l)."""
    from oracle import mixed as M  # noqa: F401
    z, x = W.water_cluster(3, W.cluster_box(3), 103)
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C = W.occupied_orbitals(S, mol.nelec // 2, 10)
    U, V = oracle.int3c(mol), oracle.int2c(mol)
    sh = np.argsort(mol.aux_l, kind="stable")
    off = np.concatenate([[0], np.cumsum(2 * mol.aux_l + 1)])
    perm = np.concatenate([np.arange(off[s], off[s + 1]) for s in sh])
    L = oracle.cholesky(V[np.ix_(perm, perm)])
    B = oracle.forward_subst(L, U[perm].reshape(len(perm), -1)).reshape(U.shape)
    X = B @ C
    naux, nao, nocc = X.shape
    npad = (naux + 127) // 128 * 128
    Xp = np.zeros((npad, nao, nocc + (nocc & 1)))
    Xp[:naux, :, :nocc] = X
    return Xp.transpose(1, 0, 2).reshape(nao, -1)


def test_mixed_mutations_break_the_device_checks():
    """Planted mistakes in the mixed formats exceed the tolerances the GPU
    tests allow between the device result and the format's exact value
    (tests/test_gpu_mixed.py) by a wide margin, so a kernel that made them
    would fail: dropping any one of the 15 kept int8 products (tolerance
    2^-39 S + 1e-13 max|K|), any one of the 11 products of the fast variant
    (2^-35 S + 1e-13 max|K|), and the hi.lo cross term of BF16x3
    (tolerance 2^-15 2 sum |x||x|, the FP32 summation bound)."""
    from oracle import mixed as M
    A = _x_rows_water3()
    K = 2 * A @ A.T
    Ke = 2 * M.int8_product(A, A)
    tight = 2.0 ** -39 * 2 * M.int8_scale_envelope(A, A) + 1e-13 * np.abs(K).max()
    assert (np.abs(Ke - K) / tight).max() < 1e3     # the format's own error, for scale
    for i in range(5):
        for j in range(5 - i):
            Km = 2 * M.int8_product(A, A, keep=lambda a, b, i=i, j=j: a + b <= 4 and (a, b) != (i, j))
            assert (np.abs(Km - Ke) / tight).max() > 4.0, (i, j)
    # the fast variant: dropping any of its 11 products breaks its tolerance
    # 2^-35 S + 1e-13 max|K|; its own error is within 2^-27 S
    Kf4 = 2 * M.int8_product(A, A, keep=M.int8_fast_keep)
    tight4 = 2.0 ** -35 * 2 * M.int8_scale_envelope(A, A) + 1e-13 * np.abs(K).max()
    assert (np.abs(Kf4 - K) / (2.0 ** -27 * 2 * M.int8_scale_envelope(A, A))).max() <= 1.0
    kept = [(i, j) for i in range(5) for j in range(5) if M.int8_fast_keep(i, j)]
    assert len(kept) == 11
    for i, j in kept:
        Km = 2 * M.int8_product(A, A, keep=lambda a, b, i=i, j=j: M.int8_fast_keep(a, b) and (a, b) != (i, j))
        assert (np.abs(Km - Kf4) / tight4).max() > 4.0, (i, j)
    hi, lo = M.split_bf16(A)
    Kf = 2 * (hi @ hi.T + hi @ lo.T + lo @ hi.T)
    ab = np.abs(hi) + np.abs(lo)
    acc = 2.0 ** -15 * 2 * (ab @ ab.T)
    Kdrop = 2 * (hi @ hi.T + lo @ hi.T)
    assert (np.abs(Kdrop - Kf) / acc).max() > 4.0


def test_int8_energy_error_decomposition_and_bound():
    """The int8 energy-error bound of dfjk_build_checked, term by term, on
    3 waters: the error of E_K = -1/2 sum_k x_k^T D x_k equals
    1/2 sum_k [2 x~^T D r + r^T D r + sum_{i+j>=5} alpha_i^T D alpha_j]
    (an identity, to FP64 rounding); each term is within its Cauchy-Schwarz
    bound in the D-seminorm; lambda bounds lambda_max(D) and R bounds the
    remainders; the assembled bound covers the actual error.  Mutations of
    the derivation (a dropped remainder term, the dropped-order sum over
    i + j >= 4) break the identity."""
    from oracle import mixed as M
    A = _x_rows_water3()
    z, x = W.water_cluster(3, W.cluster_box(3), 103)
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C = W.occupied_orbitals(S, mol.nelec // 2, 10)
    # the rows of A are (P, i) pairs with i over nocc + pad columns: expand C to match
    nao, kdim = A.shape
    D = 2 * C @ C.T
    Eex = -0.5 * np.einsum("mk,mn,nk->", A, D, A)
    Kq = 2 * M.int8_product(A, A)
    Eq = -0.25 * (D * Kq).sum()
    a, e = M.int8_slices(A)
    Ee = np.repeat(e, 256, axis=1)
    alpha = [np.ldexp(a[s], Ee - 7 * (s + 1)) for s in range(5)]
    xt = sum(alpha)
    r = A - xt
    t1 = np.einsum("mk,mn,nk->", xt, D, r)
    t2 = np.einsum("mk,mn,nk->", r, D, r)
    t3 = sum(np.einsum("mk,mn,nk->", alpha[i], D, alpha[j]) for i in range(5) for j in range(5) if i + j >= 5)
    ident = 0.5 * (2 * t1 + t2 + t3)
    tol = 1e-13 * abs(Eex)                     # FP64 rounding of the two energies
    print("identity residual %.2e, error %.2e, terms %.2e %.2e %.2e" % (abs((Eq - Eex) - ident), Eq - Eex, t1, t2, t3))
    assert abs((Eq - Eex) - ident) <= tol
    # mutations of the decomposition
    assert abs((Eq - Eex) - 0.5 * (t1 + t2 + t3)) > 3 * tol
    t3m = sum(np.einsum("mk,mn,nk->", alpha[i], D, alpha[j]) for i in range(5) for j in range(5) if i + j >= 4)
    assert abs((Eq - Eex) - 0.5 * (2 * t1 + t2 + t3m)) > 1e3 * tol
    b = M.int8_energy_bound(A, C, Eq, nsums=kdim // 256 + 16)
    lam_exact = 2 * np.linalg.eigvalsh(C.T @ C).max()
    assert lam_exact <= b["lam"] <= 1.2 * lam_exact
    assert (r ** 2).sum() <= b["R"]
    assert np.isclose(sum(b["A"]) + 0.0, sum(float((al ** 2).sum()) for al in alpha), rtol=1e-12)
    Q = np.einsum("mk,mn,nk->", xt, D, xt)
    assert Q <= b["Q"]
    assert abs(t1) <= np.sqrt(Q * b["lam"] * b["R"])
    assert abs(t2) <= b["lam"] * b["R"]
    assert abs(t3) <= b["lam"] * b["T"]
    assert abs(Eq - Eex) <= b["bound"]
    print("int8 |dE_K| %.3e, bound %.3e" % (abs(Eq - Eex), b["bound"]))


def test_int8_fast_keeps_the_diagonal_square():
    """Why the fast int8 variant keeps a_2 b_2: on 3 waters, orders i + j <= 3
    alone shift E_K by about 1e-6 Eh (the dropped a_2^2 is positive on every
    diagonal element of K), while adding a_2 b_2 back leaves an unbiased
    error 40 times below 1e-6 Eh."""
    from oracle import mixed as M
    z, x = W.water_cluster(3, W.cluster_box(3), 103)
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C = W.occupied_orbitals(S, mol.nelec // 2, 10)
    D = 2 * C @ C.T
    A = _x_rows_water3()
    EK = -0.25 * np.sum(D * (2 * A @ A.T))
    e3 = -0.25 * np.sum(D * 2 * M.int8_product(A, A, keep=lambda i, j: i + j <= 3)) - EK
    ef = -0.25 * np.sum(D * 2 * M.int8_product(A, A, keep=M.int8_fast_keep)) - EK
    assert e3 > 5e-7 and abs(ef) < 2.5e-8
