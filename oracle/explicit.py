"""Explicit Fock-space expansion of reduced MPS objects (oracle pin tier).

TEST INFRASTRUCTURE ONLY.

For a handful of orbitals the whole Fock space (times the 2S+1 states of the
singlet-embedding ghost spin) fits in memory, so every reduced object of the
spin-adapted DMRG can be expanded into ordinary many-electron vectors with
Clebsch-Gordan coefficients:
  * left block states |a, m>   from the left tensors,
  * right block states |b, m>  (orbitals to the right plus the ghost spin),
  * the two-site basis [|(a n1) j> (x) |(n2 b) j>]^0.
This gives the plain definition of the effective Hamiltonian, sigma = P^T H P x,
with H built from the unfolded one- and two-body integrals, and the explicit
matrices <alpha|O|beta> of renormalised operators.  None of the complementary
operator algebra or of the 6j/9j recoupling is used here.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import su2
from .sadmrg import LOC_N, LOC_TJ, LeftEnl, RightEnl


class Fock:
    def __init__(self, L: int):
        self.L = L
        self.dim = 4 ** L
        dets = np.arange(self.dim, dtype=np.int64)
        self.cdag = {}
        for p in range(L):
            for sg in (0, 1):
                bit = 2 * p + sg
                occ = (dets >> bit) & 1
                below = np.zeros_like(dets)
                x = dets & ((1 << bit) - 1)
                while (x != 0).any():
                    below += (x != 0)
                    x = x & (x - 1)
                src = np.nonzero(occ == 0)[0]
                dst = src | (1 << bit)
                sign = np.where(below[src] % 2 == 0, 1.0, -1.0)
                self.cdag[p, sg] = sp.csr_matrix((sign, (dst, src)), shape=(self.dim, self.dim))
        self.E = {(p, q): (self.cdag[p, 0] @ self.cdag[q, 0].T + self.cdag[p, 1] @ self.cdag[q, 1].T).tocsr()
                  for p in range(L) for q in range(L)}

    def hamiltonian(self, h, eri, e_const=0.0):
        L = self.L
        H = e_const * sp.identity(self.dim, format="csr")
        for p in range(L):
            for q in range(L):
                if h[p, q] != 0.0:
                    H = H + h[p, q] * self.E[p, q]
        for p in range(L):
            for q in range(L):
                for r in range(L):
                    for s in range(L):
                        v = eri[p, q, r, s]
                        if v == 0.0:
                            continue
                        t = self.E[p, q] @ self.E[r, s]
                        if q == r:
                            t = t - self.E[p, s]
                        H = H + 0.5 * v * t
        return H.tocsr()

    def local_creator(self, p: int, n: int, tm: int):
        """Operator string creating local state (n, m) on orbital p from empty."""
        I = sp.identity(self.dim, format="csr")
        if n == 0:
            return I
        if n == 2:
            return self.cdag[p, 0] @ self.cdag[p, 1]
        return self.cdag[p, 0] if tm == 1 else self.cdag[p, 1]


def _ms(tj):
    return list(range(-tj, tj + 1, 2))


class Expansion:
    """Explicit left/right block states of an oracle DMRG object."""

    def __init__(self, dm, fock: Fock):
        self.dm, self.F = dm, fock
        self.P = dm.P
        self.ng = self.P.twoS + 1

    def vacuum(self):
        v = np.zeros(self.F.dim)
        v[0] = 1.0
        return v

    def left_states(self, k):
        """{sector: array (d, 2j+1, Fock dim)} for the left block at bond k."""
        P, F = self.P, self.F
        cur = {(0, 0, 0): self.vacuum()[None, None, :]}
        for c in range(1, k + 1):
            E = LeftEnl(P, c, {q: v.shape[0] for q, v in cur.items()})
            U = self.dm.U[c - 1]
            nxt = {}
            for m, pcs in E.pieces.items():
                if m not in U:
                    continue
                tj = m[1]
                enl = np.zeros((E.dim[m], tj + 1, F.dim))
                for (a, n) in pcs:
                    o = E.off[(m, a, n)]
                    for ia, tma in enumerate(_ms(a[1])):
                        for tmn in _ms(LOC_TJ[n]):
                            tmm = tma + tmn
                            if abs(tmm) > tj:
                                continue
                            cgv = su2.cg(a[1], tma, LOC_TJ[n], tmn, tj, tmm)
                            if cgv == 0.0:
                                continue
                            op = F.local_creator(c - 1, n, tmn)
                            sign = (-1.0) ** (a[0] * LOC_N[n])  # P_a P_n = (-1)^{NaNn} P_n P_a
                            for r in range(cur[a].shape[0]):
                                enl[o + r, (tmm + tj) // 2] += cgv * sign * (op @ cur[a][r, ia])
                nxt[m] = np.einsum("ek,emf->kmf", U[m], enl)
            cur = nxt
        return cur

    def right_states(self, k):
        """{sector: array (d, 2j+1, Fock dim, ghost dim)} for the right block at bond k."""
        P, F = self.P, self.F
        L = P.L
        g = np.zeros((1, P.twoS + 1, F.dim, self.ng))
        for i, tm in enumerate(_ms(P.twoS)):
            g[0, i, 0, i] = 1.0
        cur = {(P.N, P.twoS, P.irrep): g}
        for c in range(L - 1, k - 1, -1):
            E = RightEnl(P, c, {q: v.shape[0] for q, v in cur.items()})
            V = self.dm.V[c]
            nxt = {}
            for m, pcs in E.pieces.items():
                if m not in V:
                    continue
                tj = m[1]
                enl = np.zeros((E.dim[m], tj + 1, F.dim, self.ng))
                for (n, b) in pcs:
                    o = E.off[(m, n, b)]
                    for ib, tmb in enumerate(_ms(b[1])):
                        for tmn in _ms(LOC_TJ[n]):
                            tmm = tmn + tmb
                            if abs(tmm) > tj:
                                continue
                            cgv = su2.cg(LOC_TJ[n], tmn, b[1], tmb, tj, tmm)
                            if cgv == 0.0:
                                continue
                            op = F.local_creator(c, n, tmn)
                            for r in range(cur[b].shape[0]):
                                enl[o + r, (tmm + tj) // 2] += cgv * (op @ cur[b][r, ib])
                nxt[m] = np.einsum("ke,emfg->kmfg", V[m], enl)
            cur = nxt
        return cur

    def two_site_basis(self, i, El, Er, secs, left_states, right_states):
        """Explicit vectors of [|(a n1) j> (x) |(n2 b) j>]^0 at step i."""
        P, F = self.P, self.F
        # enlarged left states at bond i+1 (no truncation)
        out = {}
        for m in secs:
            tj = m[1]
            lv = np.zeros((El.dim[m], tj + 1, F.dim))
            for (a, n) in El.pieces[m]:
                o = El.off[(m, a, n)]
                for ia, tma in enumerate(_ms(a[1])):
                    for tmn in _ms(LOC_TJ[n]):
                        tmm = tma + tmn
                        if abs(tmm) > tj:
                            continue
                        cgv = su2.cg(a[1], tma, LOC_TJ[n], tmn, tj, tmm)
                        if cgv == 0.0:
                            continue
                        op = F.local_creator(i, n, tmn)
                        sign = (-1.0) ** (a[0] * LOC_N[n])
                        for r in range(left_states[a].shape[0]):
                            lv[o + r, (tmm + tj) // 2] += cgv * sign * (op @ left_states[a][r, ia])
            rv = np.zeros((Er.dim[m], tj + 1, F.dim, self.ng))
            for (n, b) in Er.pieces[m]:
                o = Er.off[(m, n, b)]
                for ib, tmb in enumerate(_ms(b[1])):
                    for tmn in _ms(LOC_TJ[n]):
                        tmm = tmn + tmb
                        if abs(tmm) > tj:
                            continue
                        cgv = su2.cg(LOC_TJ[n], tmn, b[1], tmb, tj, tmm)
                        if cgv == 0.0:
                            continue
                        op = F.local_creator(i + 1, n, tmn)
                        for r in range(right_states[b].shape[0]):
                            rv[o + r, (tmm + tj) // 2] += cgv * (op @ right_states[b][r, ib])
            # singlet coupling: sum_mu <j mu; j -mu|00> |left mu> |right -mu>
            # product of a left vector (orbitals <= i) and a right vector
            # (orbitals > i): determinants combine by OR with no sign.
            basis = np.zeros((El.dim[m], Er.dim[m], F.dim * self.ng))
            for imu, tmu in enumerate(_ms(tj)):
                cgv = su2.cg(tj, tmu, tj, -tmu, 0, 0)
                jmu = (-tmu + tj) // 2
                L_ = lv[:, imu, :]  # (dl, fock)
                R_ = rv[:, jmu, :, :]  # (dr, fock, ghost)
                li = np.nonzero(np.abs(L_).sum(0))[0]
                ri = np.nonzero(np.abs(R_).sum((0, 2)))[0]
                for d1 in li:
                    for d2 in ri:
                        idx = (d1 | d2) * self.ng
                        basis[:, :, idx:idx + self.ng] += cgv * L_[:, d1][:, None, None] * R_[:, d2, :][None, :, :]
            out[m] = basis.reshape(El.dim[m] * Er.dim[m], F.dim * self.ng)
        return out


# ---------------------------------------------------------------------------
# Reduced density matrices of an MPS, written out in Fock space.  The paper's
# calc2DM (section "CheMPS2 library", the DMRG object) defines
#   Gamma_{(i s)(j t);(k s)(l t)} = <a+_{i s} a+_{j t} a_{l t} a_{k s}>,
#   Gamma^A_{ij;kl} = sum_{s t} Gamma_{(i s)(j t);(k s)(l t)},
#   Gamma^B_{ij;kl} = sum_{s t} (-1)^(s - t) Gamma_{(i s)(j t);(k s)(l t)}.
# The singlet-embedded state carries the right-boundary ghost spin; tracing it
# out leaves the average over the 2S+1 members of the multiplet, so Gamma^B
# here is that multiplet average (Gamma^A does not depend on the member).
# ---------------------------------------------------------------------------
def state_vector(ex: Expansion, dm) -> np.ndarray:
    """Normalised many-electron state (Fock dim, ghost dim) of dm's MPS at
    its current two-site centre."""
    from .sadmrg import LeftEnl, RightEnl
    P = dm.P
    i, psi = dm.center
    El = LeftEnl(P, i + 1, dm.dims[i])
    Er = RightEnl(P, i + 1, dm.dims[i + 2])
    secs = sorted(set(El.dim) & set(Er.dim))
    basis = ex.two_site_basis(i, El, Er, secs, ex.left_states(i), ex.right_states(i + 2))
    v = np.zeros(ex.F.dim * ex.ng)
    for m in secs:
        x = psi.get(m)
        if x is None:
            continue
        v += basis[m].T @ x.ravel()
    v = v.reshape(ex.F.dim, ex.ng)
    return v / np.linalg.norm(v)


def rdms_of_state(F: Fock, Psi: np.ndarray):
    """(gamma, Gamma^A, Gamma^B, <S^2>) of a normalised (Fock, ghost) state.

    Every element is an inner product of explicit vectors:
    <a+_{i s} a+_{j t} a_{l t} a_{k s}> = (a_{j t} a_{i s} Psi) . (a_{l t} a_{k s} Psi).
    <S^2> comes from the spin operators themselves, S^2 = S_- S_+ + S_z^2 + S_z,
    not from the density matrices, so that it checks them.
    """
    L = F.L
    ann = {(p, s): F.cdag[p, s].T.tocsr() for p in range(L) for s in (0, 1)}
    g1 = np.zeros((L, L))
    for s in (0, 1):
        A = np.stack([(ann[p, s] @ Psi).ravel() for p in range(L)])  # a_{p s} Psi
        g1 += A @ A.T  # <a+_{p s} a_{q s}> = (a_p Psi).(a_q Psi)
    GA = np.zeros((L, L, L, L))
    GB = np.zeros((L, L, L, L))
    for s in (0, 1):
        for t in (0, 1):
            W = np.stack([(ann[j, t] @ (ann[i, s] @ Psi)).ravel() for i in range(L) for j in range(L)])
            G = (W @ W.T).reshape(L, L, L, L)  # [i, j, k, l]
            GA += G
            GB += G if s == t else -G
    Sp = sum(F.cdag[p, 0] @ ann[p, 1] for p in range(L))
    Sz = 0.5 * sum(F.cdag[p, 0] @ ann[p, 0] - F.cdag[p, 1] @ ann[p, 1] for p in range(L))
    S2 = (Sp.T @ Sp + Sz @ Sz + Sz).tocsr()
    s2 = float(np.sum(Psi * (S2 @ Psi)))
    return g1, GA, GB, s2
