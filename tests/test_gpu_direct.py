"""Four-centre direct J/K on the GPU against the oracle's unfitted,
unscreened definitions.

* monomer, dimer and trimer: every element of J and K and both energies
  against the dense four-centre tensor (C route and D route; the trimer has
  several waves per pair class and ragged last waves);
* an 8-water cluster at a looser threshold and the 32-water cluster: sampled
  shell-pair blocks against the oracle's block routine, plus the identities
  that hold at any size (symmetry, energies as traces, K positive
  semidefinite for D = 2 C C^T, linearity in D).

Tolerance: 1e-10 of max |J| (max |K|) and 1e-10 relative on the energies
(screening at 1e-14 and FP64 rounding are far below it)."""
import numpy as np
import pytest

import oracle
import workload as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_09452_amd import dfjk as G  # noqa: E402

TOL = 1e-10


def _cluster(n, seed=1):
    if n == 1:
        z, x = W.water_monomer()
    else:
        z, x = W.water_cluster(n, W.cluster_box(n), seed)
    mol = W.make_molecule(z, x)
    C = W.occupied_orbitals(W.overlap_by_quadrature(mol), mol.nelec // 2, seed)
    return mol, C


def _plan(mol, tau=1e-14):
    return G.Plan.from_molecule(mol, schwarz_thresh=tau).screen().direct_setup()


def _np(*ts):
    return [t.cpu().numpy() for t in ts]


def _check_dense(mol, C, plan):
    D = oracle.density(C)
    Jr, Kr, EJr, EKr = oracle.exact_jk(mol, D)
    for J, K, E in (_np(*plan.direct_build(C=C)), _np(*plan.direct_build(D=D))):
        assert np.abs(J - Jr).max() <= TOL * np.abs(Jr).max()
        assert np.abs(K - Kr).max() <= TOL * np.abs(Kr).max()
        assert abs(E[0] - EJr) <= TOL * abs(EJr)
        assert abs(E[1] - EKr) <= TOL * abs(EKr)
        assert np.array_equal(J, J.T) and np.array_equal(K, K.T)


@pytest.mark.parametrize("n", [1, 2, 3])
def test_direct_dense_parity(n):
    mol, C = _cluster(n)
    plan = _plan(mol)
    st = plan.direct_stats()
    print("waters %d: pairs per class %s, quartets %d" % (n, st["pairs"], st["quartets"]))
    _check_dense(mol, C, plan)
    plan.close()


def test_direct_no_screening():
    """Threshold 0 keeps every pair and every quartet."""
    mol, C = _cluster(1)
    plan = _plan(mol, tau=0.0)
    st = plan.direct_stats()
    ns = len(mol.ao_l)
    npair = ns * (ns + 1) // 2
    assert sum(st["pairs"]) == npair
    assert st["quartets"] == npair * npair
    _check_dense(mol, C, plan)
    plan.close()


def test_direct_nonsymmetric_route_and_linearity():
    """J and K are linear in D: J(aD1 + bD2) = aJ(D1) + bJ(D2), same for K."""
    mol, C = _cluster(2)
    plan = _plan(mol)
    rng = np.random.default_rng(3)
    M = rng.standard_normal((mol.nao, mol.nao))
    D1 = oracle.density(C)
    D2 = 0.1 * (M + M.T)
    J1, K1, _ = _np(*plan.direct_build(D=D1))
    J2, K2, _ = _np(*plan.direct_build(D=D2))
    J3, K3, _ = _np(*plan.direct_build(D=0.5 * D1 - 2.0 * D2))
    assert np.abs(J3 - (0.5 * J1 - 2.0 * J2)).max() <= 1e-12 * np.abs(J3).max()
    assert np.abs(K3 - (0.5 * K1 - 2.0 * K2)).max() <= 1e-12 * np.abs(K3).max()
    Jr, Kr, _, _ = oracle.exact_jk(mol, D2)
    assert np.abs(J2 - Jr).max() <= TOL * np.abs(Jr).max()
    assert np.abs(K2 - Kr).max() <= TOL * np.abs(Kr).max()
    plan.close()


def _offsets(mol):
    return np.concatenate([[0], np.cumsum(2 * mol.ao_l + 1)])


def _check_blocks(mol, D, J, K, pairs):
    off = _offsets(mol)
    Js, Ks = oracle.exact_jk_blocks(mol, D, pairs)
    sj, sk = np.abs(J).max(), np.abs(K).max()
    for (a, c), jb, kb in zip(pairs, Js, Ks):
        assert np.abs(J[off[a]:off[a + 1], off[c]:off[c + 1]] - jb).max() <= TOL * sj, (a, c)
        assert np.abs(K[off[a]:off[a + 1], off[c]:off[c + 1]] - kb).max() <= TOL * sk, (a, c)


def _sample_pairs(mol, n, rng):
    ns = len(mol.ao_l)
    pairs = [(int(a), int(c)) for a, c in rng.integers(0, ns, (n, 2))]
    dshell = int(np.flatnonzero(mol.ao_l == 2)[0])
    pairs += [(dshell, dshell), (dshell, 0), (ns - 1, ns - 1)]
    return pairs


def _check_identities(C, J, K, E):
    D = oracle.density(C)
    assert np.array_equal(J, J.T) and np.array_equal(K, K.T)
    assert abs(E[0] - 0.5 * np.sum(D * J)) <= 1e-12 * abs(E[0])
    assert abs(E[1] + 0.25 * np.sum(D * K)) <= 1e-12 * abs(E[1])
    assert E[0] > 0 and E[1] < 0


def test_direct_eight_waters_sampled_blocks():
    mol, C = _cluster(8, seed=2)
    plan = _plan(mol, tau=1e-12)
    J, K, E = _np(*plan.direct_build(C=C))
    _check_identities(C, J, K, E)
    assert np.linalg.eigvalsh(K).min() >= -1e-10 * np.abs(K).max()
    _check_blocks(mol, oracle.density(C), J, K, _sample_pairs(mol, 12, np.random.default_rng(8)))
    plan.close()


@pytest.mark.slow
def test_direct_water32_sampled_blocks():
    z, x = W.water_cluster(32, 10.0, 1)
    mol = W.make_molecule(z, x)
    C = W.occupied_orbitals(W.overlap_by_quadrature(mol), mol.nelec // 2, 1000)
    plan = _plan(mol, tau=1e-10)
    st = plan.direct_stats()
    print("water32: pairs per class %s, quartets %d" % (st["pairs"], st["quartets"]))
    J, K, E = _np(*plan.direct_build(C=C))
    _check_identities(C, J, K, E)
    # screening at 1e-10: the dropped quartets are each below 1e-10 in size
    D = oracle.density(C)
    off = _offsets(mol)
    pairs = _sample_pairs(mol, 8, np.random.default_rng(32))
    Js, Ks = oracle.exact_jk_blocks(mol, D, pairs)
    sj, sk = np.abs(J).max(), np.abs(K).max()
    for (a, c), jb, kb in zip(pairs, Js, Ks):
        ej = np.abs(J[off[a]:off[a + 1], off[c]:off[c + 1]] - jb).max()
        ek = np.abs(K[off[a]:off[a + 1], off[c]:off[c + 1]] - kb).max()
        assert ej <= 1e-8 * sj and ek <= 1e-8 * sk, (a, c, ej / sj, ek / sk)
    plan.close()


def test_direct_delta_against_oracle():
    """Incremental build on the dimer: J0, K0 from D0, then D from perturbed
    orbitals; J, K, E against the dense exact definition for D."""
    mol, C0 = _cluster(2)
    S = W.overlap_by_quadrature(mol)
    C1 = W.perturbed_orbitals(C0, S, 1, eps=1e-2, seed=77)
    D0, D1 = oracle.density(C0), oracle.density(C1)
    plan = _plan(mol)
    J0, K0, _ = plan.direct_build(D=D0)
    J, K, E = _np(*plan.direct_build_delta(D1, D0, J0, K0))
    Jr, Kr, EJr, EKr = oracle.exact_jk(mol, D1)
    assert np.abs(J - Jr).max() <= TOL * np.abs(Jr).max()
    assert np.abs(K - Kr).max() <= TOL * np.abs(Kr).max()
    assert abs(E[0] - EJr) <= TOL * abs(EJr) and abs(E[1] - EKr) <= TOL * abs(EKr)
    assert np.array_equal(J, J.T) and np.array_equal(K, K.T)
    # D = D0 gives back J0 and K0 exactly (every quartet screened out)
    Js, Ks, _ = _np(*plan.direct_build_delta(D0, D0, J0, K0))
    assert np.array_equal(Js, J0.cpu().numpy()) and np.array_equal(Ks, K0.cpu().numpy())
    plan.close()


@pytest.mark.parametrize("eps", [1e-2, 1e-4])
def test_direct_delta_matches_full_build(eps):
    """Eight waters at tau = 1e-12: the incremental build equals the full build
    to the screening error, for a large and a small density change."""
    mol, C0 = _cluster(8, seed=2)
    S = W.overlap_by_quadrature(mol)
    C1 = W.perturbed_orbitals(C0, S, 1, eps=eps, seed=78)
    D0, D1 = oracle.density(C0), oracle.density(C1)
    plan = _plan(mol, tau=1e-12)
    J0, K0, _ = plan.direct_build(D=D0)
    Jf, Kf, Ef = _np(*plan.direct_build(D=D1))
    J, K, E = _np(*plan.direct_build_delta(D1, D0, J0, K0))
    ej = np.abs(J - Jf).max() / np.abs(Jf).max()
    ek = np.abs(K - Kf).max() / np.abs(Kf).max()
    print("eps %g: incremental vs full  J %.2e  K %.2e  dE %.2e %.2e" % (eps, ej, ek, E[0] - Ef[0], E[1] - Ef[1]))
    assert ej <= 1e-9 and ek <= 1e-9
    assert abs(E[0] - Ef[0]) <= 1e-9 * abs(Ef[0]) and abs(E[1] - Ef[1]) <= 1e-9 * abs(Ef[1])
    plan.close()


def test_direct_agrees_with_df_to_fitting_accuracy():
    """The exact J/K and the density-fitted J/K of the same molecule differ by
    the fitting error only (a sanity link between the two paths; DF energies
    lie below the exact ones, variationally)."""
    mol, C = _cluster(2)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=1e-14).screen().setup().direct_setup()
    _, _, Ed = _np(*plan.direct_build(C=C))
    _, _, Ef = _np(*plan.build(C=C))
    assert Ef[0] <= Ed[0] + 1e-12 and abs(Ef[1]) <= abs(Ed[1]) + 1e-12
    assert abs(Ef[0] - Ed[0]) <= 1e-2 * Ed[0]
    plan.close()


def test_direct_graph_replay():
    """One direct build captured in a HIP graph and replayed, with eager
    work between replays, matches the eager result each time."""
    mol, C = _cluster(2)
    plan = _plan(mol)
    Ct = torch.as_tensor(C, device="cuda")
    J0, K0, E0 = plan.direct_build(C=Ct)
    torch.cuda.synchronize()
    out = (torch.empty_like(J0), torch.empty_like(K0), torch.empty_like(E0))
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        plan.direct_build(C=Ct, out=out, stream=s)     # scratch allocated outside capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        plan.direct_build(C=Ct, out=out, stream=s)
    for _ in range(3):
        for t in out:
            t.fill_(0.0)
        g.replay()
        torch.cuda.synchronize()
        assert torch.allclose(out[0], J0, rtol=0, atol=1e-12 * float(J0.abs().max()))
        assert torch.allclose(out[1], K0, rtol=0, atol=1e-12 * float(K0.abs().max()))
        assert torch.allclose(out[2], E0, rtol=1e-12, atol=0)
        plan.direct_build(C=Ct)                         # eager work between replays
        torch.cuda.synchronize()
    plan.close()


def test_direct_errors():
    mol, C = _cluster(1)
    plan = G.Plan.from_molecule(mol)
    with pytest.raises(G.DFJKError):
        plan.direct_setup()                              # not screened
    plan.screen()
    with pytest.raises(G.DFJKError):
        plan.direct_build(C=C)                           # no tables
    plan.direct_setup()
    with pytest.raises(ValueError):
        plan.direct_build()
    with pytest.raises(ValueError):
        plan.direct_build_delta(np.zeros((2, 2)), np.zeros((2, 2)), np.zeros((2, 2)), np.zeros((2, 2)))
    with pytest.raises(ValueError):
        plan.direct_build(C=np.zeros((mol.nao + 1, 2)))
    plan.close()
