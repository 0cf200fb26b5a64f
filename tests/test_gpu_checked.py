"""dfjk_build_checked: the int8 build with a rigorous bound on its energy
error, redone in FP64 when the bound exceeds the budget.  The device's bound
is compared with the oracle's evaluation of the same formula
(oracle.mixed.int8_energy_bound, pinned term by term on the CPU), and the
result with the oracle."""
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


def case(n):
    z, x = W.water_cluster(n, W.cluster_box(n), 100 + n)
    mol = W.make_molecule(z, x)
    S = W.overlap_by_quadrature(mol)
    C = W.occupied_orbitals(S, mol.nelec // 2, 7 + n)
    return mol, S, C


def x_rows(mol, plan, C):
    """The oracle's X as int8 contraction rows (aux functions in the
    library's internal order, padded to naux_pad, columns padded to even)."""
    U, V = oracle.int3c(mol), oracle.int2c(mol)
    perm = plan.aux_order()
    L = oracle.cholesky(V[np.ix_(perm, perm)])
    B = oracle.forward_subst(L, U[perm].reshape(len(perm), -1)).reshape(U.shape)
    X = B @ C
    naux, nao, nocc = X.shape
    npad = plan.info()["naux_pad"]
    Xp = np.zeros((npad, nao, nocc + (nocc & 1)))
    Xp[:naux, :, :nocc] = X
    return Xp.transpose(1, 0, 2).reshape(nao, -1)


@pytest.mark.parametrize("n", [3, 5])
def test_checked_build_keeps_int8_within_its_bound(n):
    mol, S, C = case(n)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    J, K, E, chosen, bound = plan.build_checked(C, budget=1e-6)
    E = E.cpu().numpy()
    ref = oracle.dfjk(mol, C=C)
    assert chosen == "int8", bound
    # the bound covers the int8 error (plus the FP64 evaluation's own rounding)
    assert abs(E[1] - ref["EK"]) <= bound + 1e-10 * abs(ref["EK"])
    assert abs(E[0] - ref["EJ"]) <= 1e-10 * abs(ref["EJ"])            # J stays FP64
    # the device evaluates the same formula as the oracle on the oracle's X
    A = x_rows(mol, plan, C)
    nocc = C.shape[1]
    shape = plan.build_shape(nocc, "int8")
    kdim = shape["aux_slab"] * (nocc + (nocc & 1))
    # FP64 sums per element the library counts: the block folds of one split,
    # the split and slab partials and the reduction
    nsums = (kdim // shape["nsplit"]) // 256 + 8 + shape["nsplit"] * shape["nslab"] + 4
    b = M.int8_energy_bound(A, C, E[1], nsums=nsums)
    print("n=%d: bound device %.6e oracle %.6e, |dE_K| %.2e" % (n, bound, b["bound"], abs(E[1] - ref["EK"])))
    assert abs(bound - b["bound"]) <= 1e-6 * b["bound"]
    # the int8 K against the oracle's K within the format's bound
    Kref = ref["K"]
    assert np.abs(K.cpu().numpy() - Kref).max() <= 1e-8 * np.abs(Kref).max()
    plan.close()


def test_checked_build_falls_back_to_fp64():
    """With a budget below the bound the build is FP64, bitwise the plain
    FP64 build."""
    mol, S, C = case(3)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU).screen().setup()
    J, K, E, chosen, bound = plan.build_checked(C, budget=1e-12)
    assert chosen == "fp64" and bound > 1e-12
    J2, K2, E2 = plan.build(C=C)
    for a, b in ((J, J2), (K, K2), (E, E2)):
        assert torch.equal(a, b)
    plan.close()


def test_checked_build_over_several_slabs():
    """Aux slabs of 128 (the digit sums accumulate over the slabs): the
    result stays within its bound of the oracle."""
    mol, S, C = case(3)
    plan = G.Plan.from_molecule(mol, schwarz_thresh=TAU, aux_slab=128).screen().setup()
    assert plan.build_shape(C.shape[1], "int8")["nslab"] >= 2
    J, K, E, chosen, bound = plan.build_checked(C, budget=1e-6)
    ref = oracle.dfjk(mol, C=C)
    E = E.cpu().numpy()
    assert chosen == "int8"
    assert abs(E[1] - ref["EK"]) <= bound + 1e-10 * abs(ref["EK"])
    plan.close()
