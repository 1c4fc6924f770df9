"""CASSCF with an FCI active-space solver (oracle of the DMRG-SCF loop).

TEST INFRASTRUCTURE ONLY.  Only tests, the package smoke check and the CPU
baseline leg of the benchmark may import this module.

The paper (section "DMRG-SCF" of the library description) optimises the
orbitals of a complete-active-space wavefunction whose active-space solver is
DMRG: orbitals are split per irrep into doubly occupied (core), active and
virtual ones, the active-space energy and its 1- and 2-RDM come from the
solver, and the orbitals are updated by the augmented-Hessian Newton-Raphson
method with the exact Hessian until the orbital gradient drops below a
threshold.  Here the active-space solver is brute-force FCI (oracle.fci), so
this module is the plain definition the GPU loop is compared with.

Conventions (all real, chemist integrals g_pqrs = (pq|rs)):
  * D_pq = <E_pq>, d_pqrs = <E_pq E_rs - d_qr E_ps> = Gamma^A_{pr;qs};
    E = e_nuc + sum h_pq D_pq + 1/2 sum g_pqrs d_pqrs.
  * orbital rotation: new orbitals phi'_p = sum_q phi_q R_qp with
    R = exp(-kappa), kappa antisymmetric, kappa_pq (p > q) the parameters;
    h' = R^T h R and g' the same on every index.
  * generalised Fock F_pq = sum_m D_pm h_qm + sum_mnt d_pmnt g_qmnt; the
    gradient dE/dkappa_pq = 2 (F_pq - F_qp); the Hessian with the RDMs fixed
    (the orbital-orbital block the augmented-Hessian step uses)
      H_pq,rs = (1 - P_pq)(1 - P_rs) [2 D_pr h_qs - (F_pr + F_rp) d_qs
                                      + 2 Y_pqrs],
      Y_pqrs = sum_mn [(d_pmrn + d_pmnr) g_qmsn + d_prmn g_qsmn],
    P_pq exchanging p and q (standard second-quantised expansion of the
    energy in the rotation generators; pinned by finite differences of E).
  * non-redundant pairs: p > q in different classes (core, active, virtual)
    and in the same irrep.
  * augmented-Hessian step: the lowest eigenvector (1, x) (up to scale) of
    [[0, g^T], [g, H]]; the step x is scaled down to norm <= `max_step`.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .fci import fci_solve, rdms


def rotate(h, eri, R):
    h2 = R.T @ h @ R
    g = np.einsum("pqrs,pi->iqrs", eri, R)
    g = np.einsum("iqrs,qj->ijrs", g, R)
    g = np.einsum("ijrs,rk->ijks", g, R)
    g = np.einsum("ijks,sl->ijkl", g, R)
    return h2, g


def kappa_matrix(L, pairs, x):
    K = np.zeros((L, L))
    for (p, q), v in zip(pairs, x):
        K[p, q] = v
        K[q, p] = -v
    return K


def nonredundant_pairs(cls, orb_irrep):
    L = len(cls)
    return [(p, q) for p in range(L) for q in range(p) if cls[p] != cls[q] and orb_irrep[p] == orb_irrep[q]]


def active_hamiltonian(h, eri, core, act, e_nuc):
    """Core energy and the active-space one-body integrals with the core's
    Coulomb and exchange fields; two-body integrals restricted to the active
    orbitals."""
    e_core = e_nuc + sum(2.0 * h[c, c] for c in core)
    for c in core:
        for c2 in core:
            e_core += 2.0 * eri[c, c, c2, c2] - eri[c, c2, c2, c]
    ha = h[np.ix_(act, act)].copy()
    for c in core:
        ha += 2.0 * eri[np.ix_(act, act, [c], [c])][:, :, 0, 0] - eri[np.ix_(act, [c], [c], act)][:, 0, 0, :]
    ga = eri[np.ix_(act, act, act, act)]
    return e_core, ha, ga


def full_rdms(L, core, act, g1, G2c):
    """D and d of (closed-shell core) x (active state): g1 active 1-RDM,
    G2c active 2-RDM in chemist order (d_tuvw)."""
    D = np.zeros((L, L))
    d = np.zeros((L, L, L, L))
    for c in core:
        D[c, c] = 2.0
    D[np.ix_(act, act)] = g1
    for c in core:
        for c2 in core:
            d[c, c, c2, c2] += 4.0
            d[c, c2, c2, c] -= 2.0
    for c in core:
        for i, t in enumerate(act):
            for j, u in enumerate(act):
                d[c, c, t, u] += 2.0 * g1[i, j]
                d[t, u, c, c] += 2.0 * g1[i, j]
                d[c, u, t, c] -= g1[i, j]
                d[t, c, c, u] -= g1[i, j]
    d[np.ix_(act, act, act, act)] = G2c
    return D, d


def energy(h, eri, D, d, e_nuc=0.0):
    return e_nuc + np.einsum("pq,pq->", h, D) + 0.5 * np.einsum("pqrs,pqrs->", eri, d)


def gen_fock(h, eri, D, d):
    return D @ h.T + np.einsum("pmnt,qmnt->pq", d, eri)


def gradient(F, pairs):
    return np.array([2.0 * (F[p, q] - F[q, p]) for p, q in pairs])


def hessian(h, eri, D, d, F, pairs):
    L = h.shape[0]
    Y = (np.einsum("pmrn,qmsn->pqrs", d, eri) + np.einsum("pmnr,qmsn->pqrs", d, eri)
         + np.einsum("prmn,qsmn->pqrs", d, eri))
    delta = np.eye(L)
    FF = F + F.T

    def core_term(p, q, r, s):
        return 2.0 * D[p, r] * h[q, s] - FF[p, r] * delta[q, s] + 2.0 * Y[p, q, r, s]

    n = len(pairs)
    H = np.zeros((n, n))
    for a, (p, q) in enumerate(pairs):
        for b, (r, s) in enumerate(pairs):
            H[a, b] = (core_term(p, q, r, s) - core_term(q, p, r, s) - core_term(p, q, s, r)
                       + core_term(q, p, s, r))
    return H


def ah_step(g, H, max_step=0.5):
    n = len(g)
    A = np.zeros((n + 1, n + 1))
    A[0, 1:] = g
    A[1:, 0] = g
    A[1:, 1:] = H
    w, v = np.linalg.eigh(A)
    v0 = v[:, 0]
    x = v0[1:] / v0[0]
    nx = np.linalg.norm(x)
    if nx > max_step:
        x *= max_step / nx
    return x


class CASSCF:
    """cls[p] in {0 core, 1 active, 2 virtual}; the active orbitals are taken
    in increasing index order (the DMRG lattice order)."""

    def __init__(self, h, eri, e_nuc, N, twoS, irrep, orb_irrep, cls):
        self.h, self.eri, self.e_nuc = np.asarray(h, float), np.asarray(eri, float), float(e_nuc)
        self.L = self.h.shape[0]
        self.cls = list(cls)
        self.orb_irrep = np.asarray(orb_irrep, dtype=int)
        self.core = [p for p in range(self.L) if self.cls[p] == 0]
        self.act = [p for p in range(self.L) if self.cls[p] == 1]
        self.N, self.twoS, self.irrep = N, twoS, irrep
        self.n_act = N - 2 * len(self.core)
        self.pairs = nonredundant_pairs(self.cls, self.orb_irrep)
        ir = 0
        for c in self.core:
            ir ^= 0  # doubly occupied orbitals are totally symmetric
        self.act_irrep = irrep

    def solve_active(self, h, eri):
        e_core, ha, ga = active_hamiltonian(h, eri, self.core, self.act, self.e_nuc)
        if not self.act:
            return e_core, np.zeros((0, 0)), np.zeros((0,) * 4)
        w, v, f = fci_solve(ha, ga, self.n_act, self.twoS, self.act_irrep, self.orb_irrep[self.act])
        g1, GA = rdms(f, v[:, 0])
        return e_core + w[0], g1, np.einsum("prqs->pqrs", GA)

    def step_data(self, R):
        h, g = rotate(self.h, self.eri, R)
        e, g1, G2c = self.solve_active(h, g)
        D, d = full_rdms(self.L, self.core, self.act, g1, G2c)
        F = gen_fock(h, g, D, d)
        return e, h, g, D, d, F

    def run(self, grad_tol=1e-6, max_iter=30, max_step=0.5, R0=None):
        R = np.eye(self.L) if R0 is None else np.array(R0, float)
        hist = []
        for it in range(max_iter):
            e, h, g, D, d, F = self.step_data(R)
            grad = gradient(F, self.pairs)
            gn = float(np.linalg.norm(grad))
            hist.append((e, gn))
            if gn < grad_tol or not self.pairs:
                break
            Hs = hessian(h, g, D, d, F, self.pairs)
            x = ah_step(grad, Hs, max_step)
            R = R @ scipy.linalg.expm(-kappa_matrix(self.L, self.pairs, x))
        return hist, R
