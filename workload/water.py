"""Water-cluster workloads for the DF-J/K build.

Everything here is input preparation: geometry, basis-set tables, random
orbital coefficients and arrival times.  The basis functions are uncontracted
real spherical Gaussians; the AO overlap used to orthonormalise the occupied
orbitals is evaluated numerically (tensor Gauss-Hermite quadrature of the
function products, each function normalised by its own numerical norm), so
it shares nothing with the analytic integral code on either side.

Units: coordinates are returned in Bohr (1 Bohr = 0.529177210903 Angstrom).
"""
from __future__ import annotations

import dataclasses

import numpy as np

ANGSTROM_TO_BOHR = 1.0 / 0.529177210903

# Water monomer, Angstrom: O at the origin, H at (+-0.757, 0.587, 0).
_WATER_ANGSTROM = np.array([[0.0, 0.0, 0.0],
                            [0.757, 0.587, 0.0],
                            [-0.757, 0.587, 0.0]])
_WATER_Z = (8, 1, 1)

# AO basis per element: list of (l, exponent), uncontracted.
_AO = {
    8: [(0, 5000.0 * 0.2 ** k) for k in range(4)]
       + [(1, 20.0 * 0.3 ** k) for k in range(3)]
       + [(2, 0.8)],
    1: [(0, 20.0 * 0.2 ** k) for k in range(3)] + [(1, 0.7)],
}


def _even_tempered(alpha0, beta, counts):
    """Even-tempered auxiliary shells; each angular momentum restarts at alpha0."""
    out = []
    for l, n in enumerate(counts):
        out += [(l, alpha0 * beta ** k) for k in range(n)]
    return out


_AUX = {
    8: _even_tempered(10000.0, 0.25, (8, 5, 4, 2)),
    1: _even_tempered(50.0, 0.3, (4, 2, 1)),
}


@dataclasses.dataclass
class Molecule:
    """A molecule with its AO and auxiliary basis (one primitive per shell)."""
    charges: np.ndarray      # (natm,) int
    coords: np.ndarray       # (natm, 3) float64, Bohr
    ao_atom: np.ndarray      # (nshell,) int32
    ao_l: np.ndarray         # (nshell,) int32
    ao_exp: np.ndarray       # (nshell,) float64
    aux_atom: np.ndarray
    aux_l: np.ndarray
    aux_exp: np.ndarray

    @property
    def natm(self):
        return len(self.charges)

    @property
    def nao(self):
        return int(np.sum(2 * self.ao_l + 1))

    @property
    def naux(self):
        return int(np.sum(2 * self.aux_l + 1))

    @property
    def nelec(self):
        return int(np.sum(self.charges))


def _random_rotation(rng):
    """Haar-uniform rotation from a uniform unit quaternion."""
    q = rng.standard_normal(4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - z * w), 2 * (x * z + y * w)],
        [2 * (x * y + z * w), 1 - 2 * (x * x + z * z), 2 * (y * z - x * w)],
        [2 * (x * z - y * w), 2 * (y * z + x * w), 1 - 2 * (x * x + y * y)],
    ])


def water_monomer():
    """Atomic numbers and Bohr coordinates of one water molecule."""
    return np.array(_WATER_Z), _WATER_ANGSTROM * ANGSTROM_TO_BOHR


def water_cluster(n, box_angstrom, seed, min_oo_angstrom=2.6, max_tries=200000):
    """n rigid waters, O placed uniformly in [0, L)^3 with O-O >= min distance,
    each given a Haar-random rotation about its O.  n == 1 returns the monomer
    in its reference orientation.  Returns (charges, coords in Bohr)."""
    if n == 1:
        return water_monomer()
    rng = np.random.default_rng(seed)
    oxy = []
    tries = 0
    while len(oxy) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place %d waters in a %.1f A box" % (n, box_angstrom))
        cand = rng.uniform(0.0, box_angstrom, size=3)
        if all(np.linalg.norm(cand - o) >= min_oo_angstrom for o in oxy):
            oxy.append(cand)
    charges, coords = [], []
    for o in oxy:
        rot = _random_rotation(rng)
        for z, r in zip(_WATER_Z, _WATER_ANGSTROM):
            charges.append(z)
            coords.append(o + rot @ r)
    return np.array(charges), np.array(coords) * ANGSTROM_TO_BOHR


def make_molecule(charges, coords):
    """Attach the AO and auxiliary shells to every atom, atom by atom."""
    ao, aux = [], []
    for ia, z in enumerate(charges):
        ao += [(ia, l, e) for l, e in _AO[int(z)]]
        aux += [(ia, l, e) for l, e in _AUX[int(z)]]
    ao = np.array(ao, dtype=object)
    aux = np.array(aux, dtype=object)
    return Molecule(
        charges=np.asarray(charges, dtype=np.int64),
        coords=np.ascontiguousarray(coords, dtype=np.float64),
        ao_atom=ao[:, 0].astype(np.int32), ao_l=ao[:, 1].astype(np.int32),
        ao_exp=ao[:, 2].astype(np.float64),
        aux_atom=aux[:, 0].astype(np.int32), aux_l=aux[:, 1].astype(np.int32),
        aux_exp=aux[:, 2].astype(np.float64),
    )


# ---------------------------------------------------------------------------
# Numerical overlap (input preparation only).
# Angular shapes of the real solid harmonics, up to a constant factor per m;
# order p: (x, y, z); d: m = -2..2 -> xy, yz, 2z^2-x^2-y^2, xz, x^2-y^2.
# Each function is normalised numerically, so the constants do not matter.

def _shapes(l, x, y, z):
    if l == 0:
        return [np.ones_like(x)]
    if l == 1:
        return [x, y, z]
    if l == 2:
        return [x * y, y * z, 2 * z * z - x * x - y * y, x * z, x * x - y * y]
    if l == 3:
        return [3 * x * x * y - y ** 3, x * y * z, y * (4 * z * z - x * x - y * y),
                z * (2 * z * z - 3 * x * x - 3 * y * y), x * (4 * z * z - x * x - y * y),
                z * (x * x - y * y), x ** 3 - 3 * x * y * y]
    raise ValueError("l > 3")


_GH_T, _GH_W = np.polynomial.hermite.hermgauss(4)   # exact for degree <= 7 per axis (f x f is 6)


def _pair_raw(la, ea, A, lb, eb, B):
    """Raw overlap blocks <shape_a g_a | shape_b g_b> for many shell pairs of
    one angular class, by tensor Gauss-Hermite quadrature about the product
    centre.  A, B: (npair, 3); ea, eb: (npair,).  Returns (npair, 2la+1, 2lb+1)."""
    p = ea + eb
    P = (ea[:, None] * A + eb[:, None] * B) / p[:, None]
    s = 1.0 / np.sqrt(p)
    t = _GH_T
    w3 = (_GH_W[:, None, None] * _GH_W[None, :, None] * _GH_W[None, None, :]).ravel()
    tx, ty, tz = np.meshgrid(t, t, t, indexing="ij")
    tx, ty, tz = tx.ravel(), ty.ravel(), tz.ravel()
    # nodes r = P + t / sqrt(p), shape (npair, nnode, 3)
    r = P[:, None, :] + s[:, None, None] * np.stack([tx, ty, tz], axis=-1)[None]
    ra = r - A[:, None, :]
    rb = r - B[:, None, :]
    # integrand with the quadrature weight exp(-p|r-P|^2) divided out
    expo = (-ea[:, None] * np.sum(ra * ra, -1) - eb[:, None] * np.sum(rb * rb, -1)
            + p[:, None] * np.sum((r - P[:, None, :]) ** 2, -1))
    g = np.exp(expo)
    fa = _shapes(la, ra[..., 0], ra[..., 1], ra[..., 2])
    fb = _shapes(lb, rb[..., 0], rb[..., 1], rb[..., 2])
    out = np.empty((len(p), 2 * la + 1, 2 * lb + 1))
    vol = s ** 3
    for i, u in enumerate(fa):
        for j, v in enumerate(fb):
            out[:, i, j] = np.sum(u * v * g * w3[None, :], axis=1) * vol
    return out


def overlap_by_quadrature(mol: Molecule) -> np.ndarray:
    """AO overlap matrix of unit-normalised functions, by quadrature."""
    nsh = len(mol.ao_l)
    offs = np.concatenate([[0], np.cumsum(2 * mol.ao_l + 1)])
    A_all = mol.coords[mol.ao_atom]
    # numerical self-norms
    norms = np.empty(mol.nao)
    for l in np.unique(mol.ao_l):
        idx = np.nonzero(mol.ao_l == l)[0]
        blk = _pair_raw(l, mol.ao_exp[idx], A_all[idx], l, mol.ao_exp[idx], A_all[idx])
        for k, sh in enumerate(idx):
            norms[offs[sh]:offs[sh + 1]] = np.sqrt(np.diag(blk[k]))
    S = np.zeros((mol.nao, mol.nao))
    ia, ib = np.tril_indices(nsh)
    # pairs of distant shells overlap below 1e-300 and are skipped
    d2 = np.sum((A_all[ia] - A_all[ib]) ** 2, axis=1)
    mu = mol.ao_exp[ia] * mol.ao_exp[ib] / (mol.ao_exp[ia] + mol.ao_exp[ib])
    near = mu * d2 < 690.0
    ia, ib = ia[near], ib[near]
    for la in np.unique(mol.ao_l):
        for lb in np.unique(mol.ao_l):
            sel = (mol.ao_l[ia] == la) & (mol.ao_l[ib] == lb)
            if not np.any(sel):
                continue
            a, b = ia[sel], ib[sel]
            na, nb = 2 * la + 1, 2 * lb + 1
            for c0 in range(0, len(a), 4096):
                aa, bb = a[c0:c0 + 4096], b[c0:c0 + 4096]
                blk = _pair_raw(la, mol.ao_exp[aa], A_all[aa], lb, mol.ao_exp[bb], A_all[bb])
                rows = offs[aa][:, None] + np.arange(na)[None, :]          # (npair, na)
                cols = offs[bb][:, None] + np.arange(nb)[None, :]          # (npair, nb)
                v = blk / (norms[rows][:, :, None] * norms[cols][:, None, :])
                S[rows[:, :, None], cols[:, None, :]] = v
                S[cols[:, None, :], rows[:, :, None]] = v
    return S


def _orthonormalise(X, S):
    """C = X R^-1 with X^T S X = R^T R, so that C^T S C = I."""
    M = X.T @ S @ X
    L = np.linalg.cholesky(0.5 * (M + M.T))
    return np.linalg.solve(L, X.T).T


def occupied_orbitals(S, nocc, seed):
    """Random occupied orbitals (nao x nocc), orthonormal in the metric S."""
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((S.shape[0], nocc))
    return np.ascontiguousarray(_orthonormalise(X, S))


def perturbed_orbitals(C0, S, k, eps=1e-2, seed=1000):
    """The k-th SCF-like iterate: orth_S(C0 + eps * R_k); k == 0 returns C0."""
    if k == 0:
        return C0.copy()
    rng = np.random.default_rng(seed + k)
    R = rng.standard_normal(C0.shape)
    return np.ascontiguousarray(_orthonormalise(C0 + eps * R, S))


def poisson_stream(nreq, rate, seed, nmin=1, nmax=64):
    """Request stream: exponential inter-arrival times at `rate` per second and
    cluster sizes drawn uniformly in [nmin, nmax].  Returns (arrival_s, sizes)."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=nreq)
    sizes = rng.integers(nmin, nmax + 1, size=nreq)
    return np.cumsum(gaps), sizes


def config(name):
    """Named workloads: (n_waters, box_angstrom, geometry_seed, cocc_seed)."""
    table = {
        "water1": (1, 0.0, 0, 0),
        "water32": (32, 10.0, 1, 1),
        "water128": (128, 16.0, 4, 4),
    }
    return table[name]


def cluster_box(n):
    """Box edge (Angstrom) giving the density of 32 waters in a 10 A box."""
    return 10.0 * (n / 32.0) ** (1.0 / 3.0)


def build_case(n, box=None, geom_seed=None, cocc_seed=0):
    """Convenience: (Molecule, S, C_occ) for an n-water cluster."""
    if box is None:
        box = cluster_box(n)
    if geom_seed is None:
        geom_seed = 10000 + n
    z, xyz = water_cluster(n, box, geom_seed)
    mol = make_molecule(z, xyz)
    S = overlap_by_quadrature(mol)
    C = occupied_orbitals(S, mol.nelec // 2, cocc_seed)
    return mol, S, C


def shift_molecule(mol: Molecule, shift):
    """The same molecule rigidly translated (Bohr)."""
    return dataclasses.replace(mol, coords=mol.coords + np.asarray(shift, float)[None, :])

