"""Brute-force determinant FCI (oracle pin tier).

The paper states that the Hamiltonian together with the target spin, particle
number and point-group irrep completely determine an FCI calculation (section
"CheMPS2 library", the Problem object).  This module is that FCI, written out:

  H = E_const + sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - d_qr E_ps),
  E_pq = sum_sigma a+_{p sigma} a_{q sigma}                        (chemist ERIs)

Determinants are 2L-bit integers, bit 2p = (p, up), bit 2p+1 = (p, down); a
determinant is the product of its creators in increasing bit order acting on
the vacuum, so that the doubly occupied orbital is a+_up a+_down |0> and the
fermion order is the lattice order (the paper's local basis, section "Reduced
MPS tensors").  The spin target is imposed exactly: we work at M_S = S and add
mu * S_- S_+, which vanishes only on states of total spin S.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def _popcount_below(d: np.ndarray, bit: int) -> np.ndarray:
    mask = np.int64((1 << bit) - 1)
    x = d & mask
    c = np.zeros_like(d)
    while True:
        nz = x != 0
        if not nz.any():
            break
        c += nz
        x = x & (x - 1)
    return c


class DetSpace:
    """Determinants with fixed N and M_S (all irreps)."""

    def __init__(self, L: int, N: int, twoMs: int):
        self.L, self.N, self.twoMs = L, N, twoMs
        if (N + twoMs) % 2:
            raise ValueError("N and 2M_S parity mismatch")
        na, nb = (N + twoMs) // 2, (N - twoMs) // 2
        if na < 0 or nb < 0 or na > L or nb > L:
            self.dets = np.zeros(0, dtype=np.int64)
        else:
            dets = []
            for oa in itertools.combinations(range(L), na):
                for ob in itertools.combinations(range(L), nb):
                    d = 0
                    for p in oa:
                        d |= 1 << (2 * p)
                    for p in ob:
                        d |= 1 << (2 * p + 1)
                    dets.append(d)
            self.dets = np.array(sorted(dets), dtype=np.int64)
        self.index = {int(d): i for i, d in enumerate(self.dets)}

    def irreps(self, orb_irrep) -> np.ndarray:
        g = np.zeros(len(self.dets), dtype=np.int64)
        for p in range(self.L):
            occ = ((self.dets >> (2 * p)) & 1) + ((self.dets >> (2 * p + 1)) & 1)
            g ^= np.where(occ % 2 == 1, int(orb_irrep[p]), 0)
        return g


def hop(src: DetSpace, dst: DetSpace, p_bit: int, q_bit: int) -> sp.csr_matrix:
    """Matrix of a+_{p_bit} a_{q_bit} from src to dst (spin-orbital bits)."""
    d = src.dets
    occ_q = ((d >> q_bit) & 1) == 1
    d1 = d ^ (1 << q_bit)
    s1 = _popcount_below(d, q_bit)
    if p_bit == q_bit:
        ok = occ_q
        d2 = d
        s2 = s1  # sign applied twice cancels
        sign = np.ones(len(d))
    else:
        ok = occ_q & (((d1 >> p_bit) & 1) == 0)
        d2 = d1 | (1 << p_bit)
        s2 = _popcount_below(d1, p_bit)
        sign = np.where((s1 + s2) % 2 == 0, 1.0, -1.0)
    rows, cols, vals = [], [], []
    idx = np.nonzero(ok)[0]
    for i in idx:
        j = dst.index.get(int(d2[i]))
        if j is not None:
            rows.append(j)
            cols.append(i)
            vals.append(sign[i])
    return sp.csr_matrix((vals, (rows, cols)), shape=(len(dst.dets), len(src.dets)))


class FCI:
    """H, S_+ and E_pq in one (N, M_S = S) determinant sector."""

    def __init__(self, h, eri, N: int, twoS: int, e_const: float = 0.0):
        self.h, self.eri, self.N, self.twoS, self.e_const = h, eri, N, twoS, e_const
        L = h.shape[0]
        self.L = L
        self.space = DetSpace(L, N, twoS)
        sp_ = self.space
        self.E = {}
        for p in range(L):
            for q in range(L):
                self.E[p, q] = (hop(sp_, sp_, 2 * p, 2 * q) + hop(sp_, sp_, 2 * p + 1, 2 * q + 1)).tocsr()
        up = DetSpace(L, N, twoS + 2)
        self.Splus = None
        if len(up.dets):
            S = None
            for p in range(L):
                t = hop(sp_, up, 2 * p, 2 * p + 1)
                S = t if S is None else S + t
            self.Splus = S.tocsr()
        # one-body part with the (E E - d E) rearrangement folded in
        self.hp = h - 0.5 * np.einsum("prrs->ps", eri)

    def sigma(self, c: np.ndarray) -> np.ndarray:
        L = self.L
        D = np.stack([self.E[r, s] @ c for r in range(L) for s in range(L)])  # (L*L, dim)
        G = self.eri.reshape(L * L, L * L) @ D  # G_pq = sum_rs (pq|rs) E_rs c
        out = self.e_const * c
        for p in range(L):
            for q in range(L):
                out = out + self.E[p, q] @ (0.5 * G[p * L + q] + self.hp[p, q] * c)
        return out

    def s2_penalty(self, c: np.ndarray) -> np.ndarray:
        if self.Splus is None:
            return np.zeros_like(c)
        return self.Splus.T @ (self.Splus @ c)


def fci_solve(h, eri, N, twoS, irrep=0, orb_irrep=None, e_const=0.0, nroots=1, mu=10.0):
    """mu = 0 gives plain eigenpairs of H in the (N, M_S = S, irrep) space."""
    """Lowest `nroots` eigenpairs of total spin S, particle number N, irrep.

    Returns (energies, vectors, fci) with vectors in the full (N, M_S=S) space
    (zero outside the target irrep).
    """
    f = FCI(h, eri, N, twoS, e_const)
    L = h.shape[0]
    if orb_irrep is None:
        orb_irrep = np.zeros(L, dtype=int)
    mask = f.space.irreps(orb_irrep) == irrep
    sel = np.nonzero(mask)[0]
    n = len(sel)
    if n == 0:
        raise ValueError("empty FCI sector")

    def mv(x):
        c = np.zeros(len(f.space.dets))
        c[sel] = x
        y = f.sigma(c) + mu * f.s2_penalty(c)
        return y[sel]

    if n <= 400:
        Hm = np.stack([mv(e) for e in np.eye(n)], axis=1)
        w, v = np.linalg.eigh(0.5 * (Hm + Hm.T))
        w, v = w[:nroots], v[:, :nroots]
    else:
        op = spla.LinearOperator((n, n), matvec=mv, dtype=np.float64)
        w, v = spla.eigsh(op, k=nroots, which="SA", tol=1e-13, maxiter=20000,
                          v0=np.ones(n) / np.sqrt(n))
        o = np.argsort(w)
        w, v = w[o], v[:, o]
    vecs = np.zeros((len(f.space.dets), nroots))
    vecs[sel] = v
    # the penalty must vanish on the returned roots: they have spin exactly S
    for k in range(nroots if mu > 0 else 0):
        pen = vecs[:, k] @ f.s2_penalty(vecs[:, k])
        if pen > 1e-8:
            raise RuntimeError("spin-penalty did not isolate spin S; raise mu")
    return w, vecs, f


def rdms(f: FCI, c: np.ndarray):
    """Spin-summed 1-RDM gamma_pq = <E_pq> and the paper's Gamma^A.

    Gamma^A_{ij;kl} = sum_{sigma tau} <a+_{i s} a+_{j t} a_{l t} a_{k s}>
                    = <E_ik E_jl> - d_jk gamma_il.
    """
    L = f.L
    Ec = {pq: f.E[pq] @ c for pq in f.E}
    g1 = np.array([[c @ Ec[p, q] for q in range(L)] for p in range(L)])
    V = np.stack([Ec[p, q] for p in range(L) for q in range(L)])  # (L*L, dim)
    M = V @ V.T  # M[(k,i),(j,l)] = (E_ki c).(E_jl c) = <E_ik E_jl>
    M = M.reshape(L, L, L, L)  # [k, i, j, l]
    G = np.einsum("kijl->ijkl", M).copy()
    for j in range(L):
        G[:, j, j, :] -= g1
    return g1, G


def s2_from_gamma(gA: np.ndarray, N: int) -> float:
    """<S^2> = -N(N-4)/4 - 1/2 sum_ij Gamma^A_{ij;ji}."""
    return -N * (N - 4) / 4.0 - 0.5 * np.einsum("ijji->", gA)


def rdm_b_multiplet(f: FCI, c: np.ndarray):
    """The paper's Gamma^B_{ij;kl} = sum_{s t} (-1)^(s-t) <a+_{i s} a+_{j t}
    a_{l t} a_{k s}>, averaged over the 2S+1 members M = S .. -S of the
    multiplet of the FCI vector c (given at M = S).  The lower members are
    S_- applied to c, normalised; each expectation value is written out with
    spin-resolved hops:  Gamma^B = 4 <Sz_ik Sz_jl> - d_jk gamma_il with
    Sz_pq = (E^up_pq - E^down_pq) / 2."""
    L, N = f.L, f.N
    space, vec = f.space, c / np.linalg.norm(c)
    acc = np.zeros((L, L, L, L))
    for step in range(f.twoS + 1):
        twoM = f.twoS - 2 * step
        if step > 0:
            lower = DetSpace(L, N, twoM)
            Sm = None
            for p in range(L):
                t = hop(space, lower, 2 * p + 1, 2 * p)
                Sm = t if Sm is None else Sm + t
            vec = Sm @ vec
            vec = vec / np.linalg.norm(vec)
            space = lower
        Eu = {(p, q): hop(space, space, 2 * p, 2 * q) for p in range(L) for q in range(L)}
        Ed = {(p, q): hop(space, space, 2 * p + 1, 2 * q + 1) for p in range(L) for q in range(L)}
        Z = np.stack([0.5 * ((Eu[p, q] - Ed[p, q]) @ vec) for p in range(L) for q in range(L)])
        g1 = np.array([[vec @ ((Eu[p, q] + Ed[p, q]) @ vec) for q in range(L)] for p in range(L)])
        M = (Z @ Z.T).reshape(L, L, L, L)  # [k, i, j, l] = <Sz_ik Sz_jl>
        G = 4.0 * np.einsum("kijl->ijkl", M)
        for j in range(L):
            G[:, j, j, :] -= g1
        acc += G
    return acc / (f.twoS + 1)
