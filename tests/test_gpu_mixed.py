"""Mixed-precision K against the oracle, element by element, through the C ABI.

Each format is checked twice:
* against the format evaluated in exact arithmetic by the oracle
  (oracle.mixed, from the oracle's FP64 X), where only the device's rounding
  of the sums may differ:
    FP32, BF16x3: FP32 sums over chunks of at most 512 k folded into FP64, so
      |K - K_fmt|_{mu nu} <= 2^-15 2 sum_k |x_mu k||x_nu k| (gamma_512 in
      binary32, over the stored operands);
    INT8: the products are exact integers and only the FP64 fold rounds, so
      K equals the emulation up to FP64 rounding and a rare last-digit flip
      of a slice where the device's and the oracle's FP64 X straddle a
      rounding boundary: |K - K_emul| <= 2^-39 S + 1e-13 max|K|, S the
      scale envelope 2 sum_k 2^{e_mu(k) + e_nu(k)} (one flip moves an
      element by at most 2^-34 2^{e_mu + e_nu});
    INT8_FAST (orders i + j <= 3 and a_2 b_2): the same, but a flip of the
      last slice it uses, a_3, moves an element by up to 2^-27 2^{e_mu + e_nu}
      <= 2^-35 S: |K - K_emul| <= 2^-35 S + 1e-13 max|K|;
* against the FP64 oracle K with the format's total error bound:
    FP32 (2^-15 + 2^-23), BF16x3 (2^-15 + 2^-14) times 2 sum_k |x||x|
    (binary32 rounding 2^-24 per factor; bf16 hi + lo of a binary32 value
    within 2^-17, the dropped lo.lo below 2^-16); INT8 2^-33 S (per product
    the dropped orders and remainders stay below 2^-33 2^{e_x + e_y}),
    INT8_FAST 2^-27 S (the dropped order-4 products sum to 1.5 2^-28, the
    higher orders and remainders stay below 2^-33).
A CPU test (tests/test_oracle_pins.py) shows that dropping any one kept
product (int8) or the hi.lo cross term (BF16x3) breaks the first check.
J and E_J stay FP64 in every mode; for INT8 the energies must also be
within 1e-6 Eh of the oracle's."""
import numpy as np
import pytest

import oracle
import workload as W
from oracle import mixed as M

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_09452_amd import dfjk as G  # noqa: E402

TAU = 1e-14


def int8_pass_width(ncol):
    """Columns per pass of the half transform: at most 10 fragments of 16
    columns per pass, the fragments spread evenly over the fewest passes."""
    need = (ncol + 15) // 16
    passes = (need + 9) // 10
    return 16 * ((need + passes - 1) // passes)


def case(n, nocc=None, cseed=None):
    if n == 1:
        z, x = W.water_monomer()
    else:
        z, x = W.water_cluster(n, W.cluster_box(n), 100 + n)
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C = W.occupied_orbitals(S, nocc or mol.nelec // 2, cseed if cseed is not None else 7 + n)
    return mol, S, C


def internal_x(mol, plan, C, U=None, V=None):
    """The oracle's X_{P, mu, i} with the aux functions in the library's
    internal order (B = L^{-1} U depends on the order), padded to naux_pad."""
    U = oracle.int3c(mol) if U is None else U
    V = oracle.int2c(mol) if V is None else V
    perm = plan.aux_order()
    L = oracle.cholesky(V[np.ix_(perm, perm)])
    B = oracle.forward_subst(L, U[perm].reshape(len(perm), -1)).reshape(U.shape)
    X = B @ C
    npad = plan.info()["naux_pad"]
    Xp = np.zeros((npad,) + X.shape[1:])
    Xp[:X.shape[0]] = X
    return Xp


def int8_rows(Xp, slab):
    """Per aux slab, the rows mu of X in the int8 layout's contraction order:
    column passes (int8_pass_width), then aux rows, then the pass's columns (width
    rounded up to even, the pad column zero)."""
    npad, nao, ncol = Xp.shape
    pw = int8_pass_width(ncol)
    out = []
    for pb in range(0, npad, slab):
        Xs = Xp[pb:pb + slab]
        parts = []
        for c0 in range(0, ncol, pw):
            w = min(pw, ncol - c0)
            blk = np.zeros((Xs.shape[0], nao, w + (w & 1)))
            blk[:, :, :w] = Xs[:, :, c0:c0 + w]
            parts.append(blk.transpose(1, 0, 2).reshape(nao, -1))
        out.append(np.concatenate(parts, axis=1))
    return out


def check_format(prec, K, Kref, A_rows):
    """Both checks of the module docstring for one build; A_rows the
    per-slab contraction rows (FP64 X of the oracle)."""
    Kmax = np.abs(Kref).max()
    if prec == "int8":
        Kf = 2 * sum(M.int8_product(A, A) for A in A_rows)
        S = 2 * sum(M.int8_scale_envelope(A, A) for A in A_rows)
        tight = 2.0 ** -39 * S + 1e-13 * Kmax
        total = 2.0 ** -33 * S + 1e-12 * Kmax
    elif prec == "int8_fast":
        Kf = 2 * sum(M.int8_product(A, A, keep=M.int8_fast_keep) for A in A_rows)
        S = 2 * sum(M.int8_scale_envelope(A, A) for A in A_rows)
        tight = 2.0 ** -35 * S + 1e-13 * Kmax
        total = 2.0 ** -27 * S + 1e-12 * Kmax
    else:
        if prec == "fp32":
            ops = [(M.round_fp32(A), None) for A in A_rows]
            Kf = 2 * sum(a @ a.T for a, _ in ops)
            env = 2 * sum(np.abs(a) @ np.abs(a).T for a, _ in ops)
            ftot = 2.0 ** -15 + 2.0 ** -23
        else:
            ops = [M.split_bf16(A) for A in A_rows]
            Kf = 2 * sum(h @ h.T + h @ l.T + l @ h.T for h, l in ops)
            env = 2 * sum((np.abs(h) + np.abs(l)) @ (np.abs(h) + np.abs(l)).T for h, l in ops)
            ftot = 2.0 ** -15 + 2.0 ** -14
        absx = 2 * sum(np.abs(A) @ np.abs(A).T for A in A_rows)
        tight = 2.0 ** -15 * env + 1e-13 * Kmax
        total = ftot * absx + 1e-12 * Kmax
    r_fmt = (np.abs(K - Kf) / tight).max()
    r_tot = (np.abs(K - Kref) / total).max()
    print("%s: max|K - K_fmt|/bound %.3g  max|K - K_oracle|/bound %.3g  max|dK| %.3e"
          % (prec, r_fmt, r_tot, np.abs(K - Kref).max()))
    assert r_fmt <= 1.0
    assert r_tot <= 1.0


@pytest.fixture(scope="module")
def water3():
    mol, S, C = case(3)
    U, V = oracle.int3c(mol), oracle.int2c(mol)
    B, _ = oracle.whitened_3c(mol, U)
    ref = oracle.jk_from_B(B, C=C)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    Xp = internal_x(mol, plan, C, U, V)
    return dict(mol=mol, S=S, C=C, U=U, V=V, B=B, ref=ref, plan=plan, Xp=Xp)


@pytest.mark.parametrize("prec", ["fp32", "bf16x3", "int8", "int8_fast"])
def test_mixed_k_elementwise_against_oracle(water3, prec):
    d = water3
    J, K, E = (t.cpu().numpy() for t in d["plan"].build(C=d["C"], precision=prec))
    J64, _, E64 = (t.cpu().numpy() for t in d["plan"].build(C=d["C"]))
    assert np.array_equal(J, J64) and E[0] == E64[0]         # J and E_J stay FP64
    if prec.startswith("int8"):
        rows = int8_rows(d["Xp"], d["Xp"].shape[0])
    else:
        rows = [d["Xp"].transpose(1, 0, 2).reshape(d["Xp"].shape[1], -1)]
    check_format(prec, K, d["ref"]["K"], rows)
    dEK = abs(E[1] - d["ref"]["EK"])
    print("%s: |dE_J| %.3e |dE_K| %.3e Eh" % (prec, abs(E[0] - d["ref"]["EJ"]), dEK))
    if prec.startswith("int8"):
        assert dEK <= 1e-6 and abs(E[0] - d["ref"]["EJ"]) <= 1e-10 * abs(d["ref"]["EJ"])
    assert np.abs(K - K.T).max() == 0.0


def test_int8_several_slabs_and_a_ragged_last_slab():
    """Slabs of 128 aux rows (5 waters: four slabs, the last ragged against
    the aux count) are sliced one slab at a time."""
    mol, S, C = case(5)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU, aux_slab=128).screen().setup()
    U, V = oracle.int3c(mol), oracle.int2c(mol)
    B, _ = oracle.whitened_3c(mol, U)
    ref = oracle.jk_from_B(B, C=C)
    J, K, E = (t.cpu().numpy() for t in plan.build(C=C, precision="int8"))
    check_format("int8", K, ref["K"], int8_rows(internal_x(mol, plan, C, U, V), 128))
    assert abs(E[1] - ref["EK"]) <= 1e-6


@pytest.mark.parametrize("n,nocc", [(9, 160), (11, 291)])
def test_int8_column_passes(n, nocc):
    """160 orbitals (one pass of 160 columns, the 32-water shape) and 291
    (two passes of 160 and 131 + 1 pad columns) against the oracle; FP64 of
    the same case at 1e-10."""
    mol, S, C = case(n, nocc=nocc)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    U, V = oracle.int3c(mol), oracle.int2c(mol)
    B, _ = oracle.whitened_3c(mol, U)
    ref = oracle.jk_from_B(B, C=C)
    del B
    J, K, E = (t.cpu().numpy() for t in plan.build(C=C))
    rel = lambda a, b: np.abs(a - b).max() / np.abs(b).max()
    assert rel(J, ref["J"]) <= 1e-10 and rel(K, ref["K"]) <= 1e-10
    assert abs(E[0] - ref["EJ"]) <= 1e-10 * abs(ref["EJ"]) and abs(E[1] - ref["EK"]) <= 1e-10 * abs(ref["EK"])
    J8, K8, E8 = (t.cpu().numpy() for t in plan.build(C=C, precision="int8"))
    Xp = internal_x(mol, plan, C, U, V)
    check_format("int8", K8, ref["K"], int8_rows(Xp, Xp.shape[0]))
    assert abs(E8[1] - ref["EK"]) <= 1e-6 and np.array_equal(J8, J)


def test_int8_increment(water3):
    """K = K0 + G + G^T with G = X_U X_W^T in int8 (U = C + C0, W = C - C0):
    within the int8 bound of the increment of the oracle's K(C1)."""
    d = water3
    plan, C0 = d["plan"], d["C"]
    C1 = W.perturbed_orbitals(C0, d["S"], 1, eps=1e-2, seed=1000)
    _, K0, _ = plan.build(C=C0)
    J, K, E = (t.cpu().numpy() for t in plan.build_delta(C1, C0, K0, precision="int8"))
    r1 = oracle.jk_from_B(d["B"], C=C1)
    Xu = internal_x(d["mol"], plan, C1 + C0, d["U"], d["V"])
    Xw = internal_x(d["mol"], plan, C1 - C0, d["U"], d["V"])
    Au, Aw = int8_rows(Xu, Xu.shape[0])[0], int8_rows(Xw, Xw.shape[0])[0]
    G8 = M.int8_product(Au, Aw)
    Kf = K0.cpu().numpy() + G8 + G8.T
    S = 2 * M.int8_scale_envelope(Au, Aw)
    Kmax = np.abs(r1["K"]).max()
    assert (np.abs(K - Kf) / (2.0 ** -39 * S + 1e-13 * Kmax)).max() <= 1.0
    assert (np.abs(K - r1["K"]) / (2.0 ** -33 * S + 1e-12 * Kmax)).max() <= 1.0
    assert abs(E[1] - r1["EK"]) <= 1e-8


def test_int8_open_shell(water3):
    d = water3
    Ca = d["C"]
    Cb = W.occupied_orbitals(d["S"], 14, 102)
    ref = oracle.uks_from_B(d["B"], Ca, Cb)
    J, Ka, Kb, E = (t.cpu().numpy() for t in d["plan"].build_uks(Ca, Cb, precision="int8"))
    for Cs, Ks, Kr in ((Ca, Ka, ref["Ka"]), (Cb, Kb, ref["Kb"])):
        Xp = internal_x(d["mol"], d["plan"], Cs, d["U"], d["V"])
        A = int8_rows(Xp, Xp.shape[0])[0]
        # the open-shell K_s = X_s X_s^T carries no factor 2
        Kf = M.int8_product(A, A)
        S = M.int8_scale_envelope(A, A)
        Kmax = np.abs(Kr).max()
        assert (np.abs(Ks - Kf) / (2.0 ** -39 * S + 1e-13 * Kmax)).max() <= 1.0
        assert (np.abs(Ks - Kr) / (2.0 ** -33 * S + 1e-12 * Kmax)).max() <= 1.0
    assert abs(E[1] - ref["EK"]) <= 1e-6
