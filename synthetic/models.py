"""Seeded synthetic lattices and their analytic force constants.

This module only *builds inputs*: cells, masses, replica tables, second-order
force constants (dense, home-cell first index) and third-order force
constants (COO, home-cell first index), in the layouts of the paper's
"Interatomic Force Constants" section (FC2 is a dense 3N_b x 3N array, FC3 a
sparse COO tensor of shape 3N_b x (3N)^2).  It computes no phonon, vertex,
linewidth or conductivity quantity; both the FP64 oracle and the GPU path take
its output as their input.

Force constants come from a central pair potential
    phi(r) = k2/2 (r - r0)^2 + k3/6 (r - r0)^3,
with r0 the pair distance of the reference structure, so phi'(r0) = 0 and the
structure is a stationary point.  For a pair with separation d = r_B - r_A,
n = d/|d|, the derivatives with respect to d are
    d2phi/dd_a dd_b       = k2 n_a n_b
    d3phi/dd_a dd_b dd_c  = (k3 - 3 k2/r0) n_a n_b n_c
                            + (k2/r0) (delta_ab n_c + delta_ac n_b + delta_bc n_a)
and a displacement of atom A enters d with a minus sign, so an FC entry
carries (-1) per slot occupied by atom A.  Acoustic sum rules then hold per
pair, exactly.

Units: eV, Angstrom, amu.
"""
from __future__ import annotations

import dataclasses
import itertools

import numpy as np


@dataclasses.dataclass
class Model:
    """A periodic cell with analytic FC2 / FC3.

    lattice : (3,3) rows a1, a2, a3 in Angstrom
    frac    : (N_b,3) fractional positions of the basis atoms
    mass    : (N_b,) amu
    rep     : (n_rep,3) int32 integer replica coordinates, rep[0] == (0,0,0)
    fc2     : (3N_b, n_rep, 3N_b) eV/A^2; fc2[3i+a, l, 3j+b] = Phi(0 i a, l j b)
    fc3_i   : (nnz,) int32, 3*basis + alpha of the home-cell atom
    fc3_j   : (nnz,) int32, (rep*N_b + basis)*3 + beta
    fc3_k   : (nnz,) int32, (rep*N_b + basis)*3 + gamma
    fc3_val : (nnz,) eV/A^3
    name    : label
    params  : the readings used to build it (echoed into results)
    """

    lattice: np.ndarray
    frac: np.ndarray
    mass: np.ndarray
    rep: np.ndarray
    fc2: np.ndarray
    fc3_i: np.ndarray
    fc3_j: np.ndarray
    fc3_k: np.ndarray
    fc3_val: np.ndarray
    name: str = ""
    params: dict = dataclasses.field(default_factory=dict)

    @property
    def n_basis(self) -> int:
        return int(self.mass.shape[0])

    @property
    def n_rep(self) -> int:
        return int(self.rep.shape[0])

    @property
    def nnz(self) -> int:
        return int(self.fc3_val.shape[0])

    @property
    def volume(self) -> float:
        return float(abs(np.linalg.det(self.lattice)))


# --------------------------------------------------------------------------
# pair-potential derivative blocks
# --------------------------------------------------------------------------

def pair_fc2_block(n: np.ndarray, k2: float) -> np.ndarray:
    """d2 phi / dd dd at r = r0 (phi'(r0) = 0)."""
    return k2 * np.outer(n, n)


def pair_fc3_block(n: np.ndarray, k2: float, k3: float, r0: float) -> np.ndarray:
    """d3 phi / dd dd dd at r = r0 (phi'(r0) = 0)."""
    eye = np.eye(3)
    t = (k3 - 3.0 * k2 / r0) * np.einsum("a,b,c->abc", n, n, n)
    t += (k2 / r0) * (np.einsum("ab,c->abc", eye, n)
                      + np.einsum("ac,b->abc", eye, n)
                      + np.einsum("bc,a->abc", eye, n))
    return t


def default_replicas(extent: int = 1) -> np.ndarray:
    """Integer replica table {-extent..extent}^3 with (0,0,0) first."""
    r = range(-extent, extent + 1)
    reps = [(0, 0, 0)] + [c for c in itertools.product(r, r, r) if c != (0, 0, 0)]
    return np.asarray(reps, dtype=np.int32)


def _bonds_periodic(lattice, frac, rep, cutoff):
    """All (i, l, j, d) with |R_l + tau_j - tau_i| < cutoff, i in the home cell."""
    cart = frac @ lattice
    bonds = []
    nb = frac.shape[0]
    for i in range(nb):
        for li, l in enumerate(rep):
            R = l @ lattice
            for j in range(nb):
                if li == 0 and j == i:
                    continue
                d = R + cart[j] - cart[i]
                r = float(np.linalg.norm(d))
                if r < cutoff:
                    bonds.append((i, li, j, d))
    return bonds


def _assemble_crystal(lattice, frac, mass, rep, bond_params, cutoff, name, params):
    """Build FC2 / FC3 of a crystal from its bonds.

    bond_params(i, j, d) -> (k2, k3) or None to drop the pair.
    Every entry of FC3 keeps its full 3x3x3 Cartesian block (no pruning of
    values that cancel), with the first index in the home cell.
    """
    nb = frac.shape[0]
    nrep = rep.shape[0]
    rep_index = {tuple(int(x) for x in r): n for n, r in enumerate(rep)}
    fc2 = np.zeros((3 * nb, nrep, 3 * nb))
    fc3 = {}  # (i, (lj, j), (lk, k)) -> 3x3x3 block

    def add3(i, sj, sk, block):
        key = (i, sj, sk)
        if key in fc3:
            fc3[key] = fc3[key] + block
        else:
            fc3[key] = block.copy()

    for (i, li, j, d) in _bonds_periodic(lattice, frac, rep, cutoff):
        kk = bond_params(i, j, d)
        if kk is None:
            continue
        k2, k3 = kk
        r0 = float(np.linalg.norm(d))
        n = d / r0
        t2 = pair_fc2_block(n, k2)
        # FC2: A = (0,i), B = (l,j); sign (-1) per slot on A
        fc2[3 * i:3 * i + 3, li, 3 * j:3 * j + 3] += -t2
        fc2[3 * i:3 * i + 3, 0, 3 * i:3 * i + 3] += t2
        t3 = pair_fc3_block(n, k2, k3, r0)
        A = (0, i)
        B = (li, j)
        for s2, s3 in itertools.product((A, B), (A, B)):
            sign = -1.0  # first slot is A
            sign *= -1.0 if s2 == A else 1.0
            sign *= -1.0 if s3 == A else 1.0
            add3(i, s2, s3, sign * t3)

    keys = sorted(fc3.keys(), key=lambda k: (k[0], k[1][0], k[1][1], k[2][0], k[2][1]))
    I, J, K, V = [], [], [], []
    for (i, (lj, j), (lk, k)) in keys:
        blk = fc3[(i, (lj, j), (lk, k))]
        for a, b, c in itertools.product(range(3), range(3), range(3)):
            I.append(3 * i + a)
            J.append((lj * nb + j) * 3 + b)
            K.append((lk * nb + k) * 3 + c)
            V.append(blk[a, b, c])
    return Model(lattice=np.asarray(lattice, float), frac=np.asarray(frac, float),
                 mass=np.asarray(mass, float), rep=rep, fc2=fc2,
                 fc3_i=np.asarray(I, np.int32), fc3_j=np.asarray(J, np.int32),
                 fc3_k=np.asarray(K, np.int32), fc3_val=np.asarray(V, float),
                 name=name, params=params)


# --------------------------------------------------------------------------
# the three structures
# --------------------------------------------------------------------------

DIAMOND_A = 5.43
SI_MASS = 28.085


def diamond(a: float = DIAMOND_A, mass: float = SI_MASS, k2: float = 10.0,
            k3: float = -60.0) -> Model:
    """Diamond-structure 2-atom FCC primitive cell, nearest-neighbour springs.

    Lattice rows a1 = (0,a/2,a/2), a2 = (a/2,0,a/2), a3 = (a/2,a/2,0); atoms
    at fractional (0,0,0) and (1/4,1/4,1/4).  Replicas {-1,0,1}^3 (the 3x3x3
    supercell) hold every nearest-neighbour pair.
    """
    lat = 0.5 * a * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], float)
    frac = np.array([[0, 0, 0], [0.25, 0.25, 0.25]])
    rep = default_replicas(1)
    r_nn = a * np.sqrt(3.0) / 4.0
    cutoff = 0.5 * (r_nn + a / np.sqrt(2.0))
    return _assemble_crystal(lat, frac, np.array([mass, mass]), rep,
                             lambda i, j, d: (k2, k3), cutoff, "diamond",
                             dict(a=a, mass=mass, k2=k2, k3=k3, r0=r_nn, cutoff=cutoff))


PEROVSKITE_A = 6.3
PEROVSKITE_MASSES = (133.0, 207.0, 127.0, 127.0, 127.0)


def perovskite(seed: int = 0, a: float = PEROVSKITE_A, cutoff: float = 4.5) -> Model:
    """Cubic ABX3, 5-atom simple-cubic cell.

    A (0,0,0) 133 amu; B (1/2,1/2,1/2) 207 amu; X at (1/2,1/2,0), (1/2,0,1/2),
    (0,1/2,1/2) 127 amu.  Pairs within `cutoff` of the types A-X, B-X, X-X get
    springs (A-B, A-A, B-B excluded).  Draws: numpy default_rng(seed); first
    k2 ~ U[2,8] eV/A^2 for (A-X, B-X, X-X), then k3 ~ U[-40,-10] eV/A^3 in the
    same order.  r0 is the ideal distance of each pair.
    """
    lat = a * np.eye(3)
    frac = np.array([[0, 0, 0], [0.5, 0.5, 0.5], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]])
    species = ["A", "B", "X", "X", "X"]
    rng = np.random.default_rng(seed)
    types = ["A-X", "B-X", "X-X"]
    k2s = rng.uniform(2.0, 8.0, size=3)
    k3s = rng.uniform(-40.0, -10.0, size=3)
    table = {t: (float(k2s[n]), float(k3s[n])) for n, t in enumerate(types)}

    def bond(i, j, d):
        t = "-".join(sorted((species[i], species[j])))
        return table.get(t)

    rep = default_replicas(1)
    return _assemble_crystal(lat, frac, np.array(PEROVSKITE_MASSES), rep, bond, cutoff,
                             "perovskite",
                             dict(a=a, seed=seed, cutoff=cutoff,
                                  k2={t: table[t][0] for t in types},
                                  k3={t: table[t][1] for t in types}))


DIAMOND_CONV_BASIS = np.array([
    [0, 0, 0], [0, 0.5, 0.5], [0.5, 0, 0.5], [0.5, 0.5, 0],
    [0.25, 0.25, 0.25], [0.25, 0.75, 0.75], [0.75, 0.25, 0.75], [0.75, 0.75, 0.25]])


def glass(seed: int = 0, ncell: int = 4, a: float = DIAMOND_A, sigma_disp: float = 0.08,
          cutoff: float = 2.8, k2: float = 10.0, k3: float = -60.0,
          mass: float = SI_MASS) -> Model:
    """Disordered Gamma-point solid: displaced diamond supercell.

    ncell^3 conventional 8-atom cells (cell-major C order, then the basis order
    of DIAMOND_CONV_BASIS); displacements default_rng(seed).normal(0, sigma,
    (N,3)) Angstrom; minimum-image pairs with r < cutoff; r0 = the displaced
    distance.  Returned as a one-cell "crystal" with a single replica, so the
    first FC3 index runs over every atom.
    """
    L = ncell * a
    cells = np.array(list(itertools.product(range(ncell), range(ncell), range(ncell))), float)
    pos = (cells[:, None, :] + DIAMOND_CONV_BASIS[None, :, :]).reshape(-1, 3) * a
    rng = np.random.default_rng(seed)
    pos = pos + rng.normal(0.0, sigma_disp, size=pos.shape)
    N = pos.shape[0]
    nb3 = 3 * N
    fc2 = np.zeros((nb3, 1, nb3))
    fc3 = {}

    def add3(key, block):
        if key in fc3:
            fc3[key] = fc3[key] + block
        else:
            fc3[key] = block.copy()

    nbond = 0
    for A in range(N):
        for B in range(A + 1, N):
            d = pos[B] - pos[A]
            d -= L * np.round(d / L)
            r0 = float(np.linalg.norm(d))
            if r0 >= cutoff:
                continue
            nbond += 1
            n = d / r0
            t2 = pair_fc2_block(n, k2)
            fc2[3 * A:3 * A + 3, 0, 3 * B:3 * B + 3] += -t2
            fc2[3 * B:3 * B + 3, 0, 3 * A:3 * A + 3] += -t2
            fc2[3 * A:3 * A + 3, 0, 3 * A:3 * A + 3] += t2
            fc2[3 * B:3 * B + 3, 0, 3 * B:3 * B + 3] += t2
            t3 = pair_fc3_block(n, k2, k3, r0)
            for s1, s2, s3 in itertools.product((A, B), (A, B), (A, B)):
                sign = 1.0
                for s in (s1, s2, s3):
                    sign *= -1.0 if s == A else 1.0
                add3((s1, s2, s3), sign * t3)
    keys = sorted(fc3.keys())
    I, J, K, V = [], [], [], []
    for (x, y, z) in keys:
        blk = fc3[(x, y, z)]
        for a_, b_, c_ in itertools.product(range(3), range(3), range(3)):
            I.append(3 * x + a_)
            J.append(3 * y + b_)
            K.append(3 * z + c_)
            V.append(blk[a_, b_, c_])
    lat = L * np.eye(3)
    return Model(lattice=lat, frac=pos / L, mass=np.full(N, mass),
                 rep=np.zeros((1, 3), np.int32), fc2=fc2,
                 fc3_i=np.asarray(I, np.int32), fc3_j=np.asarray(J, np.int32),
                 fc3_k=np.asarray(K, np.int32), fc3_val=np.asarray(V, float),
                 name="glass",
                 params=dict(seed=seed, ncell=ncell, a=a, sigma_disp=sigma_disp,
                             cutoff=cutoff, k2=k2, k3=k3, mass=mass, n_bonds=nbond))


def random_cell(seed: int, n_basis: int = 2, a: float = 5.0, cutoff: float = 3.6,
                extent: int = 1) -> Model:
    """Small random crystal for tiny-input tests: FCC-like primitive lattice,
    random basis, random positive springs per pair, r0 = ideal pair distance."""
    rng = np.random.default_rng(seed)
    lat = 0.5 * a * np.array([[0, 1, 1], [1, 0, 1], [1, 1, 0]], float)
    frac = np.vstack([[0.0, 0.0, 0.0], rng.uniform(0.15, 0.85, size=(n_basis - 1, 3))])
    mass = rng.uniform(10.0, 60.0, size=n_basis)
    rep = default_replicas(extent)
    cache = {}

    def bond(i, j, d):
        key = (min(i, j), max(i, j), round(float(np.linalg.norm(d)), 6))
        if key not in cache:
            cache[key] = (float(rng.uniform(3.0, 12.0)), float(rng.uniform(-50.0, -5.0)))
        return cache[key]

    return _assemble_crystal(lat, frac, mass, rep, bond, cutoff, f"random{seed}",
                             dict(seed=seed, n_basis=n_basis, a=a, cutoff=cutoff))


def random_cluster_glass(seed: int, n_atoms: int = 8, box: float = 6.0,
                         cutoff: float = 3.4) -> Model:
    """Tiny random Gamma-point solid (periodic box), springs on pairs < cutoff."""
    rng = np.random.default_rng(seed)
    pos = rng.uniform(0.0, box, size=(n_atoms, 3))
    N = n_atoms
    fc2 = np.zeros((3 * N, 1, 3 * N))
    fc3 = {}
    for A in range(N):
        for B in range(A + 1, N):
            d = pos[B] - pos[A]
            d -= box * np.round(d / box)
            r0 = float(np.linalg.norm(d))
            if r0 >= cutoff:
                continue
            k2 = float(rng.uniform(3.0, 12.0))
            k3 = float(rng.uniform(-50.0, -5.0))
            n = d / r0
            t2 = pair_fc2_block(n, k2)
            fc2[3 * A:3 * A + 3, 0, 3 * B:3 * B + 3] += -t2
            fc2[3 * B:3 * B + 3, 0, 3 * A:3 * A + 3] += -t2
            fc2[3 * A:3 * A + 3, 0, 3 * A:3 * A + 3] += t2
            fc2[3 * B:3 * B + 3, 0, 3 * B:3 * B + 3] += t2
            t3 = pair_fc3_block(n, k2, k3, r0)
            for s in itertools.product((A, B), repeat=3):
                sign = 1.0
                for x in s:
                    sign *= -1.0 if x == A else 1.0
                fc3[s] = fc3.get(s, 0.0) + sign * t3
    I, J, K, V = [], [], [], []
    for (x, y, z) in sorted(fc3):
        blk = fc3[(x, y, z)]
        for a_, b_, c_ in itertools.product(range(3), range(3), range(3)):
            I.append(3 * x + a_)
            J.append(3 * y + b_)
            K.append(3 * z + c_)
            V.append(blk[a_, b_, c_])
    return Model(lattice=box * np.eye(3), frac=pos / box, mass=rng.uniform(10.0, 60.0, N),
                 rep=np.zeros((1, 3), np.int32), fc2=fc2,
                 fc3_i=np.asarray(I, np.int32), fc3_j=np.asarray(J, np.int32),
                 fc3_k=np.asarray(K, np.int32), fc3_val=np.asarray(V, float),
                 name=f"rglass{seed}", params=dict(seed=seed, n_atoms=n_atoms, box=box))


# --------------------------------------------------------------------------
# zone folding: crystal FCs -> Gamma-point FCs of an n1 x n2 x n3 supercell
# --------------------------------------------------------------------------

def supercell_gamma(model: Model, ns=(3, 3, 3)) -> Model:
    """Fold crystal force constants into the Gamma-point FCs of a supercell.

    Supercell atom index = cell*N_b + basis, with cells in C order over
    (c1,c2,c3) in [0,n1) x [0,n2) x [0,n3).  An entry Phi(0 i, l' j, l'' k)
    is copied, for every supercell cell c, to
    Phi((c,i), ((c+l') mod n, j), ((c+l'') mod n, k)), summing images.
    """
    n1, n2, n3 = ns
    nb = model.n_basis
    cells = np.array(list(itertools.product(range(n1), range(n2), range(n3))), np.int64)
    ncell = cells.shape[0]
    cidx = {tuple(c): n for n, c in enumerate(cells)}
    nvec = np.array(ns)
    N = ncell * nb
    fc2 = np.zeros((3 * N, 1, 3 * N))
    for c in range(ncell):
        for li, l in enumerate(model.rep):
            c2 = cidx[tuple((cells[c] + l) % nvec)]
            for i in range(nb):
                for j in range(nb):
                    fc2[3 * (c * nb + i):3 * (c * nb + i) + 3, 0,
                        3 * (c2 * nb + j):3 * (c2 * nb + j) + 3] += \
                        model.fc2[3 * i:3 * i + 3, li, 3 * j:3 * j + 3]
    acc = {}
    ia = model.fc3_i // 3
    al = model.fc3_i % 3
    jr = (model.fc3_j // 3) // nb
    jb = (model.fc3_j // 3) % nb
    be = model.fc3_j % 3
    kr = (model.fc3_k // 3) // nb
    kb = (model.fc3_k // 3) % nb
    ga = model.fc3_k % 3
    for c in range(ncell):
        cj = [cidx[tuple((cells[c] + model.rep[r]) % nvec)] for r in range(model.n_rep)]
        for e in range(model.nnz):
            I = 3 * (c * nb + ia[e]) + al[e]
            J = 3 * (cj[jr[e]] * nb + jb[e]) + be[e]
            K = 3 * (cj[kr[e]] * nb + kb[e]) + ga[e]
            acc[(I, J, K)] = acc.get((I, J, K), 0.0) + model.fc3_val[e]
    keys = sorted(acc)
    lat = model.lattice * np.array(ns)[:, None]
    frac_sc = ((cells[:, None, :] + model.frac[None, :, :]) / nvec).reshape(-1, 3)
    return Model(lattice=lat, frac=frac_sc, mass=np.tile(model.mass, ncell),
                 rep=np.zeros((1, 3), np.int32), fc2=fc2,
                 fc3_i=np.array([k[0] for k in keys], np.int32),
                 fc3_j=np.array([k[1] for k in keys], np.int32),
                 fc3_k=np.array([k[2] for k in keys], np.int32),
                 fc3_val=np.array([acc[k] for k in keys], float),
                 name=f"{model.name}_sc{n1}{n2}{n3}", params=dict(model.params, fold=ns))
