"""The 32-water cluster (960 AO, 2,784 aux, 160 occupied orbitals) against the
oracle's values in tests/golden/water32.json (written by
tests/golden/make_water32.py from the CPU oracle alone): E_J, E_K and eight
K and J rows of builds 0 and 9 of the SCF-like sequence.

FP64 must agree to 1e-10 relative (energies; rows against the largest
element of the stored rows).  The int8 mixed build must keep E_J and E_K
within 1e-6 Eh; FP32 and BF16x3 errors are printed."""
import json
import os

import numpy as np
import pytest

import workload as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2404_09452_amd import dfjk as G  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "water32.json")


@pytest.fixture(scope="module")
def water32():
    g = json.load(open(GOLDEN))
    inp = g["inputs"]
    z, xyz = W.water_cluster(inp["n_waters"], inp["box_angstrom"], inp["geometry_seed"])
    mol = W.make_molecule(z, xyz)
    S = W.overlap_by_quadrature(mol)
    C0 = W.occupied_orbitals(S, g["nocc"], inp["orbital_seed"])
    Cs = {int(k): W.perturbed_orbitals(C0, S, int(k)) for k in g["builds"]}
    plan = G.Plan.from_molecule(mol).screen().setup()
    yield g, plan, Cs
    plan.close()


def _errors(g, k, J, K, E):
    b = g["builds"][str(k)]
    rows = g["rows"]
    Kr, Jr = np.asarray(b["K_rows"]), np.asarray(b["J_rows"])
    return (abs(E[0] - b["E_J"]), abs(E[1] - b["E_K"]),
            np.abs(K[rows] - Kr).max(), np.abs(K[rows] - Kr).max() / np.abs(Kr).max(),
            np.abs(J[rows] - Jr).max() / np.abs(Jr).max(), b)


def test_water32_fp64_against_golden(water32):
    g, plan, Cs = water32
    for k, C in Cs.items():
        J, K, E = (t.cpu().numpy() for t in plan.build(C=C))
        dEJ, dEK, dK, relK, relJ, b = _errors(g, k, J, K, E)
        print("build %d fp64: |dE_J| %.2e |dE_K| %.2e  K rows rel %.2e  J rows rel %.2e" % (k, dEJ, dEK, relK, relJ))
        assert dEJ <= 1e-10 * abs(b["E_J"]) and dEK <= 1e-10 * abs(b["E_K"])
        assert relK <= 1e-10 and relJ <= 1e-10


@pytest.mark.parametrize("prec", ["int8", "int8_fast", "fp32", "bf16x3"])
def test_water32_mixed_against_golden(water32, prec):
    g, plan, Cs = water32
    for k, C in Cs.items():
        J, K, E = (t.cpu().numpy() for t in plan.build(C=C, precision=prec))
        dEJ, dEK, dK, relK, relJ, b = _errors(g, k, J, K, E)
        print("build %d %s: |dE_J| %.2e |dE_K| %.2e Eh  max|dK| (rows) %.2e" % (k, prec, dEJ, dEK, dK))
        assert relJ <= 1e-10 and dEJ <= 1e-10 * abs(b["E_J"])     # J stays FP64
        if prec.startswith("int8"):
            assert dEK <= 1e-6


def test_water32_checked_sequence(water32):
    """The ten builds of the SCF-like sequence through dfjk_build_checked
    (budget 1e-6 Eh): every build's choice and bound are reported, every
    int8 build stays within its bound of the FP64 build of the same orbitals,
    and builds 0 and 9 are within 1e-6 Eh of the oracle's stored values."""
    g, plan, Cs = water32
    inp = g["inputs"]
    z, xyz = W.water_cluster(inp["n_waters"], inp["box_angstrom"], inp["geometry_seed"])
    mol = W.make_molecule(z, xyz)
    S = W.overlap_by_quadrature(mol)
    C0 = W.occupied_orbitals(S, g["nocc"], inp["orbital_seed"])
    for k in range(10):
        C = W.perturbed_orbitals(C0, S, k)
        J, K, E, chosen, bound = plan.build_checked(C, budget=1e-6)
        E = E.cpu().numpy()
        E64 = plan.build(C=C)[2].cpu().numpy()
        print("build %d: %s, bound %.3e Eh, |E_K - E_K(fp64)| %.3e" % (k, chosen, bound, abs(E[1] - E64[1])))
        assert abs(E[0] - E64[0]) <= 1e-10 * abs(E64[0])
        if chosen == "int8":
            assert bound <= 1e-6 and abs(E[1] - E64[1]) <= bound + 1e-9
        else:
            assert bound > 1e-6 and E[1] == E64[1]
        if str(k) in g["builds"]:
            b = g["builds"][str(k)]
            assert abs(E[0] - b["E_J"]) <= 1e-6 and abs(E[1] - b["E_K"]) <= 1e-6
