"""Brute-force twin of the oracle's vertex, for tiny inputs only.

No COO grouping, no pattern or phase tables: the crystal FC3 is expanded into
a dense tensor over a periodic supercell whose size equals the q-mesh, Bloch
vectors carry their own phase e^{-i q.R_c} per supercell cell, and the vertex
is the plain triple contraction of Eq. phi3_proj,
    V(q,q1,q2) = (1/N_cells) sum_{A,B,C} Phi_sc[A,B,C]/sqrt(m_A m_B m_C)
                 u_A(q) u_B(q1) u_C(q2),   u_(c,i)(q) = eta_i(q) e^{-i q.R_c}.
Summing the first atom over every cell and dividing by their number is the
same as restricting it to the home cell when q + q1 + q2 = G.

This is test infrastructure.
"""
from __future__ import annotations

import itertools

import numpy as np

from .constants import TWO_PI


def dense_supercell_fc3(model, ns):
    """Dense Phi3 (3N x 3N x 3N) of the ns supercell, images summed."""
    n1, n2, n3 = ns
    nb = model.n_basis
    cells = np.array(list(itertools.product(range(n1), range(n2), range(n3))))
    nvec = np.array(ns)
    cidx = {tuple(c): k for k, c in enumerate(cells)}
    N3 = 3 * nb * len(cells)
    T = np.zeros((N3, N3, N3))
    ia, al = model.fc3_i // 3, model.fc3_i % 3
    jr, jb, be = (model.fc3_j // 3) // nb, (model.fc3_j // 3) % nb, model.fc3_j % 3
    kr, kb, ga = (model.fc3_k // 3) // nb, (model.fc3_k // 3) % nb, model.fc3_k % 3
    for c in range(len(cells)):
        for e in range(model.nnz):
            cj = cidx[tuple((cells[c] + model.rep[jr[e]]) % nvec)]
            ck = cidx[tuple((cells[c] + model.rep[kr[e]]) % nvec)]
            T[3 * (c * nb + ia[e]) + al[e],
              3 * (cj * nb + jb[e]) + be[e],
              3 * (ck * nb + kb[e]) + ga[e]] += model.fc3_val[e]
    return T, cells


def bloch_vectors(model, cells, ns, evec_q, qint):
    """u[(c,i,a), s] = eta_{ia}(q,s) e^{-i 2pi (qint/ns).c} / sqrt(m_i)."""
    nb = model.n_basis
    ph = np.exp(-1j * TWO_PI * (cells @ (np.asarray(qint) / np.asarray(ns, float))))
    m = np.repeat(model.mass, 3)
    u = ph[:, None, None] * (evec_q / np.sqrt(m)[:, None])[None, :, :]
    return u.reshape(len(cells) * 3 * nb, -1)


def vertex_bruteforce(model, mesh, evec):
    """V[q, q1, s, s', s''] for every (q, q1) on the mesh, q2 = -q - q1."""
    from .phonons import mesh_points
    T, cells = dense_supercell_fc3(model, mesh)
    pts = mesh_points(mesh)
    N = np.asarray(mesh)
    nq = len(pts)
    nb3 = 3 * model.n_basis
    U = [bloch_vectors(model, cells, mesh, evec[q], pts[q]) for q in range(nq)]
    out = np.zeros((nq, nq, nb3, nb3, nb3), complex)
    for q in range(nq):
        M = np.einsum("abc,as->sbc", T, U[q])          # first index contracted
        for q1 in range(nq):
            n2 = np.mod(-pts[q] - pts[q1], N)
            q2 = (n2[0] * N[1] + n2[1]) * N[2] + n2[2]
            out[q, q1] = np.einsum("sbc,bt,cu->stu", M, U[q1], U[q2]) / len(cells)
    return out


def vertex_gamma_bruteforce(model, E, mu):
    """V_mu[mu', mu''] from the dense tensor of a Gamma-point solid."""
    n3 = 3 * model.n_basis
    T = np.zeros((n3, n3, n3))
    np.add.at(T, (model.fc3_i, model.fc3_j, model.fc3_k), model.fc3_val)
    m = np.repeat(model.mass, 3)
    u = E / np.sqrt(m)[:, None]
    return np.einsum("abc,a,bt,cu->tu", T, u[:, mu], u, u)
