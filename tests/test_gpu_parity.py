"""GPU path vs the CPU oracle, element by element, through the C ABI.

Tolerances: the plain FP64 path must agree with the oracle to 1e-10 relative
(max |diff| / max |oracle|) on J and K and on E_J, E_K; per-kernel checks use
tighter bounds where the arithmetic allows (integrals 1e-12 relative plus the
screening threshold, Boys 1e-14 relative)."""
import ctypes

import numpy as np
import pytest

import oracle
import workload as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_09452_amd import _native as N  # noqa: E402
from paper_2404_09452_amd import dfjk as G  # noqa: E402

TAU = 1e-14


def rel(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / max(np.abs(np.asarray(b)).max(), 1e-300))


def case(n, seed=None, box=None):
    if n == 1:
        z, x = W.water_monomer()
    else:
        z, x = W.water_cluster(n, box or W.cluster_box(n), seed if seed is not None else 100 + n)
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C = W.occupied_orbitals(S, mol.nelec // 2, 7 + n)
    return mol, S, C


@pytest.fixture(scope="module")
def water1():
    mol, S, C = case(1)
    U = oracle.int3c(mol)
    V = oracle.int2c(mol)
    B, L = oracle.whitened_3c(mol, U)
    ref = oracle.jk_from_B(B, C=C)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    return dict(mol=mol, C=C, U=U, V=V, B=B, ref=ref, plan=plan)


def test_boys_device_matches_oracle():
    T = np.concatenate([[0.0, 1e-12, 1e-6], np.linspace(0.0, 45.0, 1801), [39.975, 39.99, 40.0, 40.01],
                        np.logspace(-3, 3, 200)])
    F = G.boys(16, T).cpu().numpy()
    ref = np.array([oracle.boys(16, t) for t in T])
    assert rel(F, ref) <= 1e-14
    relmax = float(np.max(np.abs(F - ref) / np.abs(ref)))
    assert relmax <= 5e-14, relmax


def test_int3c_water(water1):
    got = water1["plan"].export(G.EXPORT_INT3C).cpu().numpy()
    ref = water1["U"]
    assert np.all(np.abs(got - ref) <= 1e-12 * np.abs(ref).max() + 2 * TAU)


def test_metric_and_cholesky_water(water1):
    plan = water1["plan"]
    V = plan.export(G.EXPORT_METRIC).cpu().numpy()
    assert rel(V, water1["V"]) <= 1e-13
    order = plan.aux_order()
    L = plan.export(G.EXPORT_CHOL).cpu().numpy()
    Lref = oracle.cholesky(water1["V"][np.ix_(order, order)])
    assert rel(L, Lref) <= 1e-11


def test_whitened_water(water1):
    """B = L^{-1} U depends on the aux order through L: compare against the
    oracle's whitening of the metric permuted into the library's order."""
    plan = water1["plan"]
    order = plan.aux_order()
    got = plan.export(G.EXPORT_B).cpu().numpy()
    Lref = oracle.cholesky(water1["V"][np.ix_(order, order)])
    U = water1["U"][order]
    Bref = oracle.forward_subst(Lref, U.reshape(U.shape[0], -1)).reshape(U.shape)
    assert rel(got, Bref) <= 1e-11


def test_jk_water_c_route(water1):
    J, K, E = water1["plan"].build(C=water1["C"])
    ref = water1["ref"]
    J, K, E = J.cpu().numpy(), K.cpu().numpy(), E.cpu().numpy()
    assert rel(J, ref["J"]) <= 1e-10
    assert rel(K, ref["K"]) <= 1e-10
    assert abs(E[0] - ref["EJ"]) <= 1e-10 * abs(ref["EJ"])
    assert abs(E[1] - ref["EK"]) <= 1e-10 * abs(ref["EK"])


def test_jk_water_d_route(water1):
    D = oracle.density(water1["C"])
    J, K, E = water1["plan"].build(D=D)
    ref = water1["ref"]
    assert rel(J.cpu().numpy(), ref["J"]) <= 1e-10
    assert rel(K.cpu().numpy(), ref["K"]) <= 1e-10
    E = E.cpu().numpy()
    assert abs(E[1] - ref["EK"]) <= 1e-10 * abs(ref["EK"])


def test_build_is_bitwise_deterministic(water1):
    a = [t.cpu().numpy().copy() for t in water1["plan"].build(C=water1["C"])]
    b = [t.cpu().numpy().copy() for t in water1["plan"].build(C=water1["C"])]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("n", [2, 3, 5])
def test_jk_clusters(n):
    """Several tiles and ragged tails: nao = 30 n, naux = 87 n."""
    mol, S, C = case(n)
    ref = oracle.dfjk(mol, C=C)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    J, K, E = (t.cpu().numpy() for t in plan.build(C=C))
    assert rel(J, ref["J"]) <= 1e-10
    assert rel(K, ref["K"]) <= 1e-10
    assert abs(E[0] - ref["EJ"]) <= 1e-10 * abs(ref["EJ"])
    assert abs(E[1] - ref["EK"]) <= 1e-10 * abs(ref["EK"])


@pytest.fixture(scope="module")
def cluster3_seq():
    mol, S, C0 = case(3)
    C1 = W.perturbed_orbitals(C0, S, 1, eps=1e-2, seed=1000)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    _, K0, _ = plan.build(C=C0)
    ref = [t.cpu().numpy() for t in plan.build(C=C1)]
    return dict(mol=mol, C0=C0, C1=C1, plan=plan, K0=K0, ref=ref)


def test_delta_build_fp64_reproduces_direct_build(cluster3_seq):
    """K0 + G + G^T with G = X_U X_W^T in FP64 equals K(D) built directly."""
    d = cluster3_seq
    J, K, E = (t.cpu().numpy() for t in d["plan"].build_delta(d["C1"], d["C0"], d["K0"], precision="fp64"))
    J1, K1, E1 = d["ref"]
    assert np.array_equal(J, J1)
    assert rel(K, K1) <= 1e-12
    assert abs(E[1] - E1[1]) <= 1e-12 * abs(E1[1])
    # and against the oracle for D(C1)
    r = oracle.dfjk(d["mol"], C=d["C1"])
    assert rel(K, r["K"]) <= 1e-10


@pytest.mark.parametrize("prec", ["fp32", "int8"])
def test_increment_is_invariant_to_the_orbital_gauge(cluster3_seq, prec):
    """Orbitals with one column's sign flipped and two columns rotated into each
    other give the same density; the increment rotates C onto C0 first, so its
    error stays that of the small step (without the alignment W = C - C0 would
    be O(1) and the error that of a direct mixed build)."""
    d = cluster3_seq
    plan, C1 = d["plan"], d["C1"]
    Cg = C1.copy()
    Cg[:, 0] *= -1.0
    c, s_ = np.cos(0.7), np.sin(0.7)
    a, b = Cg[:, 1].copy(), Cg[:, 2].copy()
    Cg[:, 1], Cg[:, 2] = c * a - s_ * b, s_ * a + c * b
    J1, K1, E1 = d["ref"]
    _, Kp, Ep = (t.cpu().numpy() for t in plan.build_delta(C1, d["C0"], d["K0"], precision=prec))
    Jg, Kg, Eg = (t.cpu().numpy() for t in plan.build_delta(Cg, d["C0"], d["K0"], precision=prec))
    _, Km, Em = (t.cpu().numpy() for t in plan.build(C=C1, precision=prec))
    err_p, err_g, err_direct = abs(Ep[1] - E1[1]), abs(Eg[1] - E1[1]), abs(Em[1] - E1[1])
    print("%s: |dE_K| aligned-step %.3e  gauge-changed %.3e  direct %.3e" % (prec, err_p, err_g, err_direct))
    assert rel(Jg, J1) <= 1e-12                               # J comes from D itself
    assert err_g <= 4.0 * err_p + 1e-11
    assert rel(Kg, K1) <= 4.0 * rel(Kp, K1) + 1e-12
    if prec == "fp32":
        assert err_g <= 0.2 * err_direct


@pytest.mark.parametrize("prec", ["fp32", "bf16x3"])
def test_delta_build_mixed_error_shrinks_with_the_step(cluster3_seq, prec):
    d = cluster3_seq
    J1, K1, E1 = d["ref"]
    _, Kd, Ed = (t.cpu().numpy() for t in d["plan"].build_delta(d["C1"], d["C0"], d["K0"], precision=prec))
    _, Km, Em = (t.cpu().numpy() for t in d["plan"].build(C=d["C1"], precision=prec))
    err_delta, err_direct = abs(Ed[1] - E1[1]), abs(Em[1] - E1[1])
    print("%s: |dE_K| direct %.3e  incremental %.3e" % (prec, err_direct, err_delta))
    assert Ed[0] == E1[0]
    assert err_delta <= 0.05 * err_direct + 1e-12
    assert np.abs(Kd - Kd.T).max() == 0.0


@pytest.fixture(scope="module")
def cluster5():
    mol, S, C = case(5)
    ref = oracle.dfjk(mol, C=C)
    one = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    return dict(mol=mol, S=S, C=C, ref=ref, one=one,
                base=[t.cpu().numpy() for t in one.build(C=C)])


@pytest.mark.parametrize("slab", [128, 384])
def test_aux_slabs_match_one_slab(cluster5, slab):
    """Streaming the K build over aux slabs (naux_pad 512: 4 slabs, or 384 + a ragged 128)
    changes only the order of the split-K sum."""
    d = cluster5
    plan = G.Plan.from_molecule(d["mol"], schwarz_thresh=TAU, aux_slab=slab).screen().setup().profile()
    assert plan.info()["naux_pad"] == 512
    J, K, E = (t.cpu().numpy() for t in plan.build(C=d["C"]))
    nslab = (512 + slab - 1) // slab
    assert plan.profile_read()["build.halftransform"][1] == nslab
    J1, K1, E1 = d["base"]
    assert np.array_equal(J, J1)
    assert rel(K, K1) <= 1e-13
    assert abs(E[1] - E1[1]) <= 1e-13 * abs(E1[1])
    assert rel(K, d["ref"]["K"]) <= 1e-10
    # density route through the same slabs
    D = 2.0 * d["C"] @ d["C"].T
    _, KD, ED = (t.cpu().numpy() for t in plan.build(D=D))
    assert rel(KD, d["ref"]["K"]) <= 1e-10
    # mixed and incremental builds keep their error bounds across slabs
    _, Km, Em = (t.cpu().numpy() for t in plan.build(C=d["C"], precision="fp32"))
    assert abs(Em[1] - E1[1]) <= 1e-5 * abs(E1[1])
    C1 = W.perturbed_orbitals(d["C"], d["S"], 1, eps=1e-2, seed=1000)
    K0 = d["one"].build(C=d["C"])[1]
    _, Kd, Ed = (t.cpu().numpy() for t in plan.build_delta(C1, d["C"], K0, precision="fp64"))
    _, Kr, Er = (t.cpu().numpy() for t in d["one"].build(C=C1))
    assert rel(Kd, Kr) <= 1e-12


@pytest.mark.parametrize("n,nb", [(1, 4), (1, 0), (3, 14)])
def test_uks_against_oracle(n, nb):
    """Open-shell build: alpha = the occupied orbitals, beta = nb columns of a
    second orthonormal set (0: no beta electrons)."""
    mol, S, Ca = case(n)
    Cb = W.occupied_orbitals(S, max(nb, 1), 99 + n)[:, :nb]
    ref = oracle.dfjk_uks(mol, Ca, Cb)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    J, Ka, Kb, E = (t.cpu().numpy() for t in plan.build_uks(Ca, Cb))
    assert rel(J, ref["J"]) <= 1e-10
    assert rel(Ka, ref["Ka"]) <= 1e-10
    if nb:
        assert rel(Kb, ref["Kb"]) <= 1e-10
    else:
        assert np.all(Kb == 0.0)
    assert abs(E[0] - ref["EJ"]) <= 1e-10 * abs(ref["EJ"])
    assert abs(E[1] - ref["EK"]) <= 1e-10 * abs(ref["EK"])
    # mixed-precision exchange, FP64 J
    J32, Ka32, Kb32, E32 = (t.cpu().numpy() for t in plan.build_uks(Ca, Cb, precision="fp32"))
    assert np.array_equal(J32, J) and E32[0] == E[0]
    assert abs(E32[1] - E[1]) <= 1e-5 * abs(E[1])


def test_uks_closed_shell_matches_rks(cluster5):
    d = cluster5
    J, Ka, Kb, E = (t.cpu().numpy() for t in d["one"].build_uks(d["C"], d["C"]))
    J1, K1, E1 = d["base"]
    assert np.array_equal(Ka, Kb)
    assert rel(2.0 * Ka, K1) <= 1e-13
    assert rel(J, J1) <= 1e-13
    assert abs(E[1] - E1[1]) <= 1e-13 * abs(E1[1])


@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "int8"])
def test_build_replays_in_a_hip_graph(cluster3_seq, prec):
    """A whole build captured once in a HIP graph and replayed with new orbitals
    written into the captured input: every replay equals an eager build bitwise
    (eager builds and synchronisations run between the replays)."""
    d = cluster3_seq
    plan = d["plan"]
    C0 = torch.as_tensor(d["C0"], device="cuda")
    C1 = torch.as_tensor(d["C1"], device="cuda")
    nao, nocc = C0.shape
    Cbuf = C0.clone()
    out = (torch.empty((nao, nao), dtype=torch.float64, device="cuda"),
           torch.empty((nao, nao), dtype=torch.float64, device="cuda"),
           torch.empty(2, dtype=torch.float64, device="cuda"))
    plan.build(C=Cbuf, precision=prec, out=out)           # scratch allocated outside the capture
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.build(C=Cbuf, precision=prec, out=out)
    torch.cuda.synchronize()
    for C in (C1, C0, C1, C1):
        Cbuf.copy_(C)
        g.replay()
        torch.cuda.synchronize()
        got = [t.cpu().numpy().copy() for t in out]
        ref = [t.cpu().numpy() for t in plan.build(C=C, precision=prec)]
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


@pytest.fixture(scope="module")
def batch_set():
    cases = [case(1), case(2), case(3), case(5)]
    plans = [G.Plan.from_molecule(m, schwarz_thresh=TAU).screen().setup() for m, _, _ in cases]
    # the monomer appears twice, with two different orbital sets
    S1 = cases[0][1]
    cases.append((cases[0][0], S1, W.occupied_orbitals(S1, 5, 1234)))
    plans.append(plans[0])
    return cases, plans


@pytest.mark.parametrize("prec", ["fp64", "bf16x3", "int8", "int8_fast"])
def test_batch_matches_single_builds(batch_set, prec):
    cases, plans = batch_set
    Cs = [C for _, _, C in cases]
    batch = G.Batch(plans, [C.shape[1] for C in Cs], precision=prec)
    outs = batch.build(Cs)
    torch.cuda.synchronize()
    for (mol, _, C), plan, (J, K, E) in zip(cases, plans, outs):
        J1, K1, E1 = (t.cpu().numpy() for t in plan.build(C=C, precision=prec))
        J, K, E = J.cpu().numpy(), K.cpu().numpy(), E.cpu().numpy()
        assert np.array_equal(J, J1) and E[0] == E1[0]
        if prec == "fp64":
            # only the split-K summation order differs from the single build
            assert rel(K, K1) <= 1e-13
            assert abs(E[1] - E1[1]) <= 1e-13 * abs(E1[1])
        else:
            # the batch contracts one aux slab where a single build may use two
            # (overlapped), which moves the FP32 chunk boundaries (int8: the
            # scale blocks, at the 2^-33 truncation level)
            tol = 1e-9 if prec.startswith("int8") else 1e-6
            assert rel(K, K1) <= tol
            assert abs(E[1] - E1[1]) <= tol * abs(E1[1])
    if prec == "fp64":   # one molecule against the oracle
        mol, _, C = cases[2]
        ref = oracle.dfjk(mol, C=C)
        assert rel(outs[2][1].cpu().numpy(), ref["K"]) <= 1e-10


def test_batch_with_mixed_tile_widths(batch_set):
    """A batch whose molecules' K tiles differ (plans forced to 128-, 64- and
    96-wide tiles and one left to the rule) beside a molecule that needs
    several aux slabs (not grouped): the grouped syrk launches per width and
    the grouped reduction with per-molecule widths give each molecule its
    single build's J bitwise and K up to the split-K order."""
    cases, _ = batch_set
    uniq = cases[:4] + [cases[2]]
    plans = [G.Plan.from_molecule(m, schwarz_thresh=TAU, k_tile=kt).screen().setup()
             for (m, _, _), kt in zip(uniq[:4], (128, 64, 96, 0))]
    # and one molecule on 128-wide aux slabs (several slabs: its own path in the batch)
    plans.append(G.Plan.from_molecule(uniq[4][0], schwarz_thresh=TAU, aux_slab=128).screen().setup())
    assert plans[-1].build_shape(uniq[4][2].shape[1])["nslab"] > 1
    Cs = [C for _, _, C in uniq]
    outs = G.Batch(plans, [C.shape[1] for C in Cs]).build(Cs)
    torch.cuda.synchronize()
    for plan, C, (J, K, E) in zip(plans, Cs, outs):
        J1, K1, E1 = (t.cpu().numpy() for t in plan.build(C=C))
        assert np.array_equal(J.cpu().numpy(), J1)
        assert rel(K.cpu().numpy(), K1) <= 1e-13
        assert abs(E.cpu().numpy()[1] - E1[1]) <= 1e-13 * abs(E1[1])
    mol, _, C = uniq[0]
    ref = oracle.dfjk(mol, C=C)
    assert rel(outs[0][1].cpu().numpy(), ref["K"]) <= 1e-10
    for plan in plans:
        plan.close()


def test_setup_batch_matches_single_setups(batch_set):
    """dfjk_setup_batch on uneven molecules (1, 2, 3 and 5 waters) and on 18
    plans (more than one grouped launch per integral class): the three-centre
    integrals, the factor, B and the builds of every plan equal those of its
    own dfjk_setup bitwise, and one molecule matches the oracle."""
    cases, plans = batch_set
    uniq, singles = cases[:4], plans[:4]
    fresh = G.setup_batch([G.Plan.from_molecule(m, schwarz_thresh=TAU).screen() for m, _, _ in uniq])
    for (mol, _, C), one, plan in zip(uniq, singles, fresh):
        for kind in (G.EXPORT_INT3C, G.EXPORT_CHOL, G.EXPORT_B):
            assert torch.equal(plan.export(kind), one.export(kind)), (mol.nao, kind)
        for prec in ("fp64", "int8"):
            J1, K1, E1 = (t.cpu().numpy() for t in one.build(C=C, precision=prec))
            J2, K2, E2 = (t.cpu().numpy() for t in plan.build(C=C, precision=prec))
            assert np.array_equal(J1, J2) and np.array_equal(K1, K2) and np.array_equal(E1, E2)
    mol, _, C = uniq[2]
    ref = oracle.dfjk(mol, C=C)
    J, K, _ = (t.cpu().numpy() for t in fresh[2].build(C=C))
    assert rel(K, ref["K"]) <= 1e-10 and rel(J, ref["J"]) <= 1e-10
    many = G.setup_batch([G.Plan.from_molecule(uniq[i % 3][0], schwarz_thresh=TAU).screen() for i in range(18)])
    for i, plan in enumerate(many):
        assert torch.equal(plan.export(G.EXPORT_B), singles[i % 3].export(G.EXPORT_B)), i
    for plan in fresh + many:
        plan.close()


def test_setup_batch_rejects_a_repeated_plan(batch_set):
    _, plans = batch_set
    p = G.Plan.from_molecule(batch_set[0][0][0], schwarz_thresh=TAU).screen()
    with pytest.raises(G.DFJKError) as e:
        G.setup_batch([p, p])
    assert e.value.status == "INVALID" and "twice" in e.value.message
    p.close()


def test_batch_replays_in_a_hip_graph(batch_set):
    cases, plans = batch_set
    Cs = [torch.as_tensor(C, device="cuda") for _, _, C in cases]
    bufs = [C.clone() for C in Cs]
    batch = G.Batch(plans, [C.shape[1] for C in Cs])
    outs = batch.build(bufs)
    torch.cuda.synchronize()
    ref = [[t.cpu().numpy().copy() for t in o] for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.build(bufs, outs=outs)
    for rep in range(3):
        for o in outs:
            for t in o:
                t.fill_(float("nan"))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            for t, x in zip(o, r):
                assert np.array_equal(t.cpu().numpy(), x)


def test_build_host_convenience(water1):
    """Host arrays in, host arrays out: the same J, K, E as the plan path."""
    mol, C = water1["mol"], water1["C"]
    J, K, E = G.build_host(mol.coords, mol.ao_atom, mol.ao_l, mol.ao_exp, mol.aux_atom, mol.aux_l, mol.aux_exp,
                           C=C, schwarz_thresh=TAU)
    J1, K1, E1 = (t.cpu().numpy() for t in water1["plan"].build(C=C))
    assert np.array_equal(J, J1) and np.array_equal(K, K1) and np.array_equal(E, E1)
    D = 2.0 * C @ C.T
    _, KD, _ = G.build_host(mol.coords, mol.ao_atom, mol.ao_l, mol.ao_exp, mol.aux_atom, mol.aux_l, mol.aux_exp,
                            D=D, schwarz_thresh=TAU)
    assert rel(KD, water1["ref"]["K"]) <= 1e-10


@pytest.mark.parametrize("nocc", [1, 30])
def test_occupation_extremes(water1, nocc):
    """One occupied column (single-fragment half transform) and every AO
    occupied (nocc = nao)."""
    mol = water1["mol"]
    S = W.overlap_by_quadrature(mol)
    C = W.occupied_orbitals(S, nocc, 11)
    ref = oracle.jk_from_B(water1["B"], C=C)
    J, K, E = (t.cpu().numpy() for t in water1["plan"].build(C=C))
    assert rel(J, ref["J"]) <= 1e-10 and rel(K, ref["K"]) <= 1e-10
    assert abs(E[1] - ref["EK"]) <= 1e-10 * abs(ref["EK"])


def test_density_route_with_column_passes():
    """Nine waters through the density route: X has nao = 270 columns, more than
    one 256-column pass of the half transform."""
    mol, S, C = case(9)
    D = 2.0 * C @ C.T
    ref = oracle.dfjk(mol, D=D)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    J, K, E = (t.cpu().numpy() for t in plan.build(D=D))
    assert rel(J, ref["J"]) <= 1e-10 and rel(K, ref["K"]) <= 1e-10
    assert abs(E[1] - ref["EK"]) <= 1e-10 * abs(ref["EK"])


def test_zero_threshold_keeps_every_pair(water1):
    """Threshold 0 keeps every shell pair and triplet (the unscreened definition)."""
    mol, C = water1["mol"], water1["C"]
    plan = G.Plan.from_molecule(mol, schwarz_thresh=0.0).screen().setup()
    inf = plan.info()
    assert inf["sig_shell_pairs"] == inf["nshell_pairs"]
    assert inf["triplets_kept"] == inf["nshell_pairs"] * len(mol.aux_l)
    J, K, E = (t.cpu().numpy() for t in plan.build(C=C))
    assert rel(K, water1["ref"]["K"]) <= 1e-11
    assert rel(J, water1["ref"]["J"]) <= 1e-11


@pytest.mark.parametrize("slab", [128, 384])
def test_host_resident_B_matches_device_B(cluster5, slab):
    """B moved to page-locked host memory and streamed back slab by slab:
    K and the energies equal the device-resident build with the same slabs,
    J to the order of its slab sums."""
    d = cluster5
    dev = G.Plan.from_molecule(d["mol"], schwarz_thresh=TAU, aux_slab=slab).screen().setup()
    host = G.Plan.from_molecule(d["mol"], schwarz_thresh=TAU, aux_slab=slab).screen().setup().offload()
    C1 = W.perturbed_orbitals(d["C"], d["S"], 2, eps=1e-2, seed=1000)
    for C in (d["C"], C1):                      # a second build reuses the staging buffers
        for prec in ("fp64", "fp32"):
            J1, K1, E1 = (t.cpu().numpy() for t in dev.build(C=C, precision=prec))
            J2, K2, E2 = (t.cpu().numpy() for t in host.build(C=C, precision=prec))
            assert np.array_equal(K1, K2)
            assert np.array_equal(E1, E2)
            assert rel(J2, J1) <= 1e-13
    J, K, E = (t.cpu().numpy() for t in host.build(C=d["C"]))
    assert rel(K, d["ref"]["K"]) <= 1e-10 and rel(J, d["ref"]["J"]) <= 1e-10
    with pytest.raises(G.DFJKError) as e:
        host.export(G.EXPORT_B)
    assert e.value.status == "STATE"
    with pytest.raises(G.DFJKError) as e:
        host.build(D=2.0 * d["C"] @ d["C"].T)
    assert e.value.status == "UNSUPPORTED"
    host.close()
    dev.close()


@pytest.mark.parametrize("slab", [0, 128])
def test_setup_straight_into_host_memory(cluster5, slab):
    """dfjk_setup_host under a device budget far below B: U and B formed in
    row blocks, each block's rows copied into the host slabs.  The host B
    equals the one dfjk_offload copies from a whole setup (every row of B is
    the same GEMM row), so builds in every precision are bitwise those of the
    offloaded plan, and FP64 matches the oracle.  The whole setup forms
    L^-1 block row by block row on its side stream beside the factor, the
    row-block setup after the whole factor: equal builds also show that
    both orders give the same L^-1."""
    d = cluster5
    ref_plan = G.Plan.from_molecule(d["mol"], schwarz_thresh=TAU, aux_slab=slab).screen().setup().offload()
    plan = G.Plan.from_molecule(d["mol"], schwarz_thresh=TAU, aux_slab=slab).screen()
    info = plan.info()
    nf_pad, npad = -(-info["nf"] // 64) * 64, info["naux_pad"]
    b_bytes = nf_pad * npad * 8
    hb, db = ctypes.c_size_t(), ctypes.c_size_t()
    assert N.lib().dfjk_setup_host_bytes(plan._h, 0, ctypes.byref(hb), ctypes.byref(db)) == 0
    fixed = db.value - 3 * b_bytes                        # all but the U and two B row buffers
    rows = max(nf_pad // 16, 32)
    budget = fixed + 3 * rows * npad * 8 + 8192           # about nf/16 rows per block
    plan.setup_host(max_device_bytes=budget)
    dev_bytes = plan.setup_host_info["device_bytes"]
    print("nf %d, B %.2f MB, device workspace %.2f MB (budget %.2f MB)"
          % (info["nf"], b_bytes / 1e6, dev_bytes / 1e6, budget / 1e6))
    assert dev_bytes <= budget and dev_bytes < b_bytes
    C1 = W.perturbed_orbitals(d["C"], d["S"], 2, eps=1e-2, seed=1000)
    for C in (d["C"], C1):
        for prec in ("fp64", "int8", "fp32"):
            J1, K1, E1 = (t.cpu().numpy() for t in ref_plan.build(C=C, precision=prec))
            J2, K2, E2 = (t.cpu().numpy() for t in plan.build(C=C, precision=prec))
            assert np.array_equal(J1, J2) and np.array_equal(K1, K2) and np.array_equal(E1, E2), prec
    J, K, E = (t.cpu().numpy() for t in plan.build(C=d["C"]))
    assert rel(K, d["ref"]["K"]) <= 1e-10 and rel(J, d["ref"]["J"]) <= 1e-10
    with pytest.raises(G.DFJKError) as e:
        plan.setup_host()
    assert e.value.status == "STATE"
    plan.close()
    ref_plan.close()


def test_setup_host_refuses_a_budget_below_one_pair(cluster5):
    plan = G.Plan.from_molecule(cluster5["mol"], schwarz_thresh=TAU).screen()
    with pytest.raises(G.DFJKError) as e:
        plan.setup_host(max_device_bytes=1 << 20)
    assert e.value.status == "OOM"
    plan.close()


@pytest.mark.parametrize("n,tile", [(3, 64), (5, 64), (3, 96), (5, 96), (3, 128), (5, 128)])
def test_k_tile_choices(n, tile):
    """The FP64 syrk, its partials and reduction on 64-, 96- and 128-wide
    tiles (ragged last tile row: nao 90 and 150), C and density routes,
    against the oracle."""
    mol, S, C = case(n)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU, k_tile=tile).screen().setup()
    shape = plan.build_shape(C.shape[1])
    assert shape["k_tile"] == tile and shape["nsplit"] >= 1 and shape["nslab"] == 1
    J, K, E = (t.cpu().numpy() for t in plan.build(C=C))
    ref = oracle.dfjk(mol, C=C)
    assert rel(K, ref["K"]) <= 1e-10 and rel(J, ref["J"]) <= 1e-10
    assert abs(E[1] - ref["EK"]) <= 1e-10 * abs(ref["EK"])
    J2, K2, E2 = (t.cpu().numpy() for t in plan.build(D=oracle.density(C)))
    assert rel(K2, ref["K"]) <= 1e-10
    plan.close()


def test_autotuned_split_count(cluster5):
    """The autotuner keeps one of its candidates; builds then use it and still
    agree with the oracle."""
    d = cluster5
    plan = G.Plan.from_molecule(d["mol"], schwarz_thresh=TAU).screen().setup()
    chosen, times = plan.autotune(d["C"])
    assert chosen in times and len(times) >= 2 and all(t > 0 for t in times.values())
    shape = plan.build_shape(d["C"].shape[1])
    assert (shape["k_tile"], shape["nsplit"]) == chosen
    print("split candidates (ms per build):", times, "chosen", chosen)
    J, K, E = (t.cpu().numpy() for t in plan.build(C=d["C"]))
    assert rel(K, d["ref"]["K"]) <= 1e-10
    J2, K2, E2 = (t.cpu().numpy() for t in plan.build(C=d["C"]))
    assert np.array_equal(K, K2)
    plan.close()
