"""Write water32.json: oracle values for the 32-water cluster (test fixture).

Calls only the CPU oracle (oracle.dfjk_streamed: unscreened Coulomb-metric
density fitting evaluated one slice of auxiliary shells at a time) and the
seeded input generator.  The cluster is 32 waters in a 10 Angstrom box,
geometry seed 1 (960 AO, 2,784 aux); the orbitals are 160 random occupied
orbitals (seed 1) and the SCF-like iterates C_k = orth_S(C_0 + 1e-2 R_k)
with R_k seeded 1000 + k.  The file holds E_J and E_K of builds 0 and 9,
the K and J rows of eight seeded AO indices (seed 32) for both builds.

Run from the repository root:  python tests/golden/make_water32.py
(a few minutes on eight cores, about 20 GB of memory).
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workload as W  # noqa: E402

BUILDS = (0, 9)
ROW_SEED = 32
NROWS = 8


def main(out=os.path.join(HERE, "water32.json")):
    t0 = time.time()
    n, box, gseed, cseed = W.config("water32")
    z, xyz = W.water_cluster(n, box, gseed)
    mol = W.make_molecule(z, xyz)
    S = W.overlap_by_quadrature(mol)
    nocc = mol.nelec // 2
    C0 = W.occupied_orbitals(S, nocc, cseed)
    Cs = [W.perturbed_orbitals(C0, S, k) for k in BUILDS]
    rows = np.sort(np.random.default_rng(ROW_SEED).choice(mol.nao, NROWS, replace=False))
    print("water32: nao %d naux %d nocc %d" % (mol.nao, mol.naux, nocc), flush=True)
    res = oracle.dfjk_streamed(mol, Cs, rows)
    for k, r in zip(BUILDS, res):
        print("build %d: E_J %.12f E_K %.12f" % (k, r["E_J"], r["E_K"]))
    doc = {
        "what": "oracle J/K of the 32-water cluster, unscreened Coulomb-metric density fitting, "
                "builds 0 and 9 of the SCF-like orbital sequence",
        "generator": "tests/golden/make_water32.py (oracle.dfjk_streamed)",
        "inputs": {"n_waters": n, "box_angstrom": box, "geometry_seed": gseed, "orbital_seed": cseed,
                   "perturbation": "C_k = orth_S(C_0 + 1e-2 R_k), R_k seeded 1000 + k",
                   "row_seed": ROW_SEED},
        "nao": mol.nao, "naux": mol.naux, "nocc": nocc,
        "rows": [int(r) for r in rows],
        "builds": {str(k): {"E_J": r["E_J"], "E_K": r["E_K"],
                            "K_rows": r["K_rows"].tolist(), "J_rows": r["J_rows"].tolist()}
                   for k, r in zip(BUILDS, res)},
    }
    with open(out, "w") as f:
        json.dump(doc, f, separators=(",", ":"))
    print("wrote %s (%.1fs)" % (out, time.time() - t0))


if __name__ == "__main__":
    main()
