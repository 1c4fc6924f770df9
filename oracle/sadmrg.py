"""Plain FP64 spin-adapted two-site DMRG (the oracle).

TEST INFRASTRUCTURE ONLY.  Only tests, the package smoke check and the CPU
baseline leg of the benchmark may import this module.

What it follows in the paper (arXiv:1312.2415):
  * MPS ansatz, canonical forms, two-site micro-iteration, Davidson, SVD with
    truncation to the D largest reduced singular values, sweeping
    (section "DMRG for ab initio quantum chemistry").
  * Complementary operators: one-body integrals folded into the two-body ones
    with 1/(N-1) (trick (a)), bare renormalized operators with one or two
    second-quantized operators on a side (trick (b)), complementary operators
    with two, three or four operators on a side built by summing integrals
    over the common indices (trick (c)), storage of only one of O and O^dagger
    (trick (d)) -- section "Complementary operators".
  * SU(2) x U(1) x P symmetry with reduced (Wigner-Eckart) tensors, the local
    basis labels, singlet embedding at the right boundary, and the doublet
    operators b+ = a+, b_s = (-1)^(1/2-s) a_{-s} -- section "Symmetry-adapted
    DMRG", eqs. tensordecomp, creaannih1/2.
  * kappa normalisation and discarded weight -- eqs. for kappa and w^disc.

Readings where the paper is silent:
  * The two-site object is kept in the "TT" coupling of the paper's StoTT
    equation (left block (x) site i coupled to the middle bond spin j_M, site
    i+1 (x) right block coupled to the same j_M, the pair coupled to a singlet
    with the right-boundary "ghost" spin S_G of singlet embedding).  In this
    basis H_eff is symmetric in the plain inner product and the SVD acts
    directly per (j_M, N_M, I_M) group.
  * H_eff is applied through two enlarged blocks X = (left block + site i) and
    Y = (site i+1 + right block), with complementary operators on the larger
    side for the pair terms.  Reduced elements of coupled products are taken
    from Clebsch-Gordan sums (oracle.su2), never from 6j/9j formulas.
  * Truncation ranks by kappa = s / sqrt(2 j_M + 1) (the paper's lambda up to
    a global factor), stable, ties broken by sector order then index.

Conventions: spins doubled (tj = 2j).  A sector label is (N, tj, G) where N is
the number of electrons to the LEFT of the bond and G their irrep, for left
and right blocks alike.  Local multiplets n = 0 (empty), 1 (single, s=1/2),
2 (double).  Fermion order = lattice order, doubly occupied = a+_up a+_down.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from . import su2

SQ2 = math.sqrt(2.0)
SQ3 = math.sqrt(3.0)
LOC_N = (0, 1, 2)
LOC_TJ = (0, 1, 0)


def loc_irrep(n: int, g: int) -> int:
    return g if n == 1 else 0


# ---------------------------------------------------------------------------
# Site (one-orbital) reduced operators: dict (n', n) -> value
# ---------------------------------------------------------------------------
@dataclass
class SOp:
    tk: int
    dN: int
    odd: bool
    el: dict


SITE_I = SOp(0, 0, False, {(0, 0): 1.0, (1, 1): 1.0, (2, 2): 1.0})
# <s||b+||e> = 1, <d||b+||s> = -sqrt2 ; <e||b||s> = -sqrt2, <s||b||d> = -1
SITE_CDAG = SOp(1, 1, True, {(1, 0): 1.0, (2, 1): -SQ2})
SITE_C = SOp(1, -1, True, {(0, 1): -SQ2, (1, 2): -1.0})


def sprod(U: SOp, V: SOp, tK: int) -> SOp:
    """Reduced elements of the same-site product [U x V]^K (V acts first)."""
    el = {}
    for (n2, n1), v in V.el.items():
        for (n3, n2b), u in U.el.items():
            if n2b != n2:
                continue
            c = su2.same_space_coupling(LOC_TJ[n1], LOC_TJ[n2], LOC_TJ[n3], U.tk, V.tk, tK)
            if c != 0.0:
                el[(n3, n1)] = el.get((n3, n1), 0.0) + c * u * v
    el = {k: v for k, v in el.items() if abs(v) > 1e-15}
    return SOp(tK, U.dN + V.dN, U.odd ^ V.odd, el)


SITE_A0 = sprod(SITE_CDAG, SITE_CDAG, 0)            # [b+ b+]^0
SITE_B = {0: sprod(SITE_CDAG, SITE_C, 0), 2: sprod(SITE_CDAG, SITE_C, 2)}  # [b+ b]^j, keyed by 2j
SITE_AA0 = sprod(SITE_C, SITE_C, 0)                 # [b b]^0
SITE_E = SOp(0, 0, False, {k: -SQ2 * v for k, v in SITE_B[0].el.items()})  # E_kk = -sqrt2 [b+ b]^0
SITE_CDAG_E = sprod(SITE_CDAG, SITE_E, 1)           # b+ E_kk
SITE_E_C = sprod(SITE_E, SITE_C, 1)                 # E_kk b


def site_h(w_kkkk: float) -> SOp:
    # 1/2 W_kkkk sum_{st} a+_s a+_t a_t a_s = W_kkkk n_up n_down
    return SOp(0, 0, False, {(2, 2): w_kkkk})


# ---------------------------------------------------------------------------
# Block operators
# ---------------------------------------------------------------------------
@dataclass
class Op:
    tk: int
    dN: int
    dG: int
    odd: bool
    blocks: dict = field(default_factory=dict)  # (bra_label, ket_label) -> ndarray

    def add(self, key, mat):
        if key in self.blocks:
            self.blocks[key] = self.blocks[key] + mat
        else:
            self.blocks[key] = mat.copy()


def zero_like(tk, dN, dG, odd):
    return Op(tk, dN, dG, odd, {})


def adjoint(op: Op) -> Op:
    """The conjugate tensor Tbar_q = (-1)^(k-q) (T_{-q})^dagger.

    <j||Tbar||j'> = (-1)^(j'+k-j) sqrt((2j'+1)/(2j+1)) <j'||T||j>.
    """
    out = Op(op.tk, -op.dN, op.dG, op.odd, {})
    for (bra, ket), m in op.blocks.items():
        tjp, tj = bra[1], ket[1]  # old bra j', old ket j ; new bra = old ket
        e = (tjp + op.tk - tj)
        assert e % 2 == 0
        f = (-1) ** (e // 2) * math.sqrt((tjp + 1) / (tj + 1))
        out.blocks[(ket, bra)] = f * m.T
    return out


def lincomb(terms, tk, dN, dG, odd) -> Op:
    out = Op(tk, dN, dG, odd, {})
    for c, op in terms:
        if c == 0.0 or op is None:
            continue
        assert op.tk == tk and op.dN == dN and op.odd == odd, "incompatible ops in lincomb"
        for key, m in op.blocks.items():
            out.add(key, c * m)
    return out


def scale(op: Op, c: float) -> Op:
    return Op(op.tk, op.dN, op.dG, op.odd, {k: c * m for k, m in op.blocks.items()})


def plus_transpose(op: Op) -> Op:
    """op + op^T for a rank-0 operator (its Hermitian-conjugate partner)."""
    assert op.tk == 0 and op.dN == 0
    out = Op(0, 0, op.dG, op.odd, {})
    for (bra, ket), m in op.blocks.items():
        out.add((bra, ket), m)
        out.add((ket, bra), m.T)
    return out


# ---------------------------------------------------------------------------
# Problem and symmetry sectors
# ---------------------------------------------------------------------------
class Problem:
    def __init__(self, h, eri, N, twoS, irrep=0, orb_irrep=None, e_const=0.0):
        h = np.asarray(h, dtype=np.float64)
        eri = np.asarray(eri, dtype=np.float64)
        self.L = L = h.shape[0]
        self.N, self.twoS, self.irrep = int(N), int(twoS), int(irrep)
        self.orb_irrep = np.zeros(L, dtype=int) if orb_irrep is None else np.asarray(orb_irrep, dtype=int)
        self.e_const = float(e_const)
        if self.N < 2:
            raise ValueError("the one-body folding needs N >= 2")
        if self.N > 2 * L or (self.N - self.twoS) % 2 or self.twoS > self.N or self.twoS < 0:
            raise ValueError("inconsistent (N, S)")
        self.h, self.eri = h, eri
        # paper, section "Complementary operators", trick (a): fold the one-body
        # integrals into the two-body ones (written here in chemist order):
        # W_pqrs = (pq|rs) + [h_pq d_rs + h_rs d_pq] / (N - 1)
        d = np.eye(L)
        self.W = eri + (np.einsum("pq,rs->pqrs", h, d) + np.einsum("rs,pq->pqrs", h, d)) / (self.N - 1)

    def mode_left(self, k):
        """Left block at bond k holds bare pairs iff it is the smaller side."""
        return "bare" if k <= self.L - k else "compl"

    def mode_right(self, k):
        return "bare" if self.L - k < k else "compl"


def left_multiplicities(P: Problem):
    out = [{(0, 0, 0): 1}]
    for k in range(P.L):
        nxt = {}
        for (N, tj, G), c in out[-1].items():
            for n in range(3):
                g2 = G ^ loc_irrep(n, P.orb_irrep[k])
                for tj2 in range(abs(tj - LOC_TJ[n]), tj + LOC_TJ[n] + 1, 2):
                    key = (N + LOC_N[n], tj2, g2)
                    nxt[key] = nxt.get(key, 0) + c
        out.append(nxt)
    return out


def right_multiplicities(P: Problem):
    """Multiplets of (orbitals k..L-1) + ghost spin S_G, labelled by bond k."""
    out = [None] * (P.L + 1)
    out[P.L] = {(P.N, P.twoS, P.irrep): 1}
    for k in range(P.L - 1, -1, -1):
        nxt = {}
        for (Nb, tjb, Gb), c in out[k + 1].items():
            for n in range(3):
                N = Nb - LOC_N[n]
                if N < 0:
                    continue
                G = Gb ^ loc_irrep(n, P.orb_irrep[k])
                for tj in range(abs(tjb - LOC_TJ[n]), tjb + LOC_TJ[n] + 1, 2):
                    key = (N, tj, G)
                    nxt[key] = nxt.get(key, 0) + c
        out[k] = nxt
    return out


def fci_caps(P: Problem):
    lm, rm = left_multiplicities(P), right_multiplicities(P)
    caps = []
    for k in range(P.L + 1):
        c = {}
        for key, v in lm[k].items():
            if key in rm[k]:
                c[key] = min(v, rm[k][key])
        caps.append(dict(sorted(c.items())))
    return caps


def distribute(D: int, caps: dict) -> dict:
    """Split D equally over the sectors, capped by the FCI dimensions.

    Paper, section "DMRG": the virtual dimension is distributed equally over all
    symmetry sectors without exceeding the FCI dimension.  Reading: visit the
    sectors by ascending cap (ties by label), give each min(cap, floor(rest /
    sectors left)); then hand out the remainder one by one in label order to
    sectors still below their cap.
    """
    labels = sorted(caps)
    if sum(caps.values()) <= D:
        return dict(caps)
    order = sorted(labels, key=lambda q: (caps[q], q))
    dims, rest, left = {}, D, len(order)
    for q in order:
        d = min(caps[q], rest // left)
        dims[q] = d
        rest -= d
        left -= 1
    while rest > 0:
        moved = False
        for q in labels:
            if rest == 0:
                break
            if dims[q] < caps[q]:
                dims[q] += 1
                rest -= 1
                moved = True
        if not moved:
            break
    return {q: dims[q] for q in labels if dims[q] > 0}


# ---------------------------------------------------------------------------
# Enlarged bases
# ---------------------------------------------------------------------------
class LeftEnl:
    """Left block at bond c-1 (x) site c-1, coupled block-first, at bond c."""

    def __init__(self, P: Problem, c: int, left_dims: dict, keep=None):
        g = P.orb_irrep[c - 1]
        self.pieces, self.dim = {}, {}
        for a in sorted(left_dims):
            Na, tja, Ga = a
            for n in range(3):
                for tjm in range(abs(tja - LOC_TJ[n]), tja + LOC_TJ[n] + 1, 2):
                    m = (Na + LOC_N[n], tjm, Ga ^ loc_irrep(n, g))
                    if keep is not None and m not in keep:
                        continue
                    self.pieces.setdefault(m, []).append((a, n))
        self.pieces = dict(sorted(self.pieces.items()))
        self.off = {}
        for m, pcs in self.pieces.items():
            o = 0
            for (a, n) in pcs:
                self.off[(m, a, n)] = o
                o += left_dims[a]
            self.dim[m] = o
        self.sub = left_dims


class RightEnl:
    """Site c (x) right block at bond c+1, coupled site-first, at bond c."""

    def __init__(self, P: Problem, c: int, right_dims: dict, keep=None):
        g = P.orb_irrep[c]
        self.pieces, self.dim = {}, {}
        for n in range(3):
            for b in sorted(right_dims):
                Nb, tjb, Gb = b
                for tjm in range(abs(tjb - LOC_TJ[n]), tjb + LOC_TJ[n] + 1, 2):
                    m = (Nb - LOC_N[n], tjm, Gb ^ loc_irrep(n, g))
                    if m[0] < 0:
                        continue
                    if keep is not None and m not in keep:
                        continue
                    self.pieces.setdefault(m, []).append((n, b))
        self.pieces = dict(sorted(self.pieces.items()))
        self.off = {}
        for m, pcs in self.pieces.items():
            o = 0
            for (n, b) in pcs:
                self.off[(m, n, b)] = o
                o += right_dims[b]
            self.dim[m] = o
        self.sub = right_dims


def couple_left(out: Op, X: Op, s: SOp, E: LeftEnl, coef: float):
    """out += coef * [X x s]^K in the left enlarged basis (K = out.tk).

    Sign (-1)^(parity(s) * N_a): the site operator passes the block's electrons.
    """
    if coef == 0.0:
        return
    tK = out.tk
    idx = {}
    for m, pcs in E.pieces.items():
        for (a, n) in pcs:
            idx.setdefault((a, n), []).append(m)
    for (abra, aket), xm in X.blocks.items():
        for (nb, nk), sv in s.el.items():
            for mk in idx.get((aket, nk), ()):
                for mb in idx.get((abra, nb), ()):
                    if not su2.triangle(mk[1], tK, mb[1]):
                        continue
                    c9 = su2.product_coupling(aket[1], LOC_TJ[nk], mk[1], X.tk, s.tk, tK,
                                              abra[1], LOC_TJ[nb], mb[1])
                    if c9 == 0.0:
                        continue
                    sign = -1.0 if (s.odd and aket[0] % 2) else 1.0
                    key = (mb, mk)
                    if key not in out.blocks:
                        out.blocks[key] = np.zeros((E.dim[mb], E.dim[mk]))
                    ob, ok = E.off[(mb, abra, nb)], E.off[(mk, aket, nk)]
                    out.blocks[key][ob:ob + xm.shape[0], ok:ok + xm.shape[1]] += coef * c9 * sign * sv * xm


def couple_right(out: Op, s: SOp, Y: Op, E: RightEnl, coef: float):
    """out += coef * [s x Y]^K in the right enlarged basis.

    Sign (-1)^(parity(Y) * N_n): the block operator passes the site electrons.
    """
    if coef == 0.0:
        return
    tK = out.tk
    idx = {}
    for m, pcs in E.pieces.items():
        for (n, b) in pcs:
            idx.setdefault((n, b), []).append(m)
    for (bbra, bket), ym in Y.blocks.items():
        for (nb, nk), sv in s.el.items():
            for mk in idx.get((nk, bket), ()):
                for mb in idx.get((nb, bbra), ()):
                    if not su2.triangle(mk[1], tK, mb[1]):
                        continue
                    c9 = su2.product_coupling(LOC_TJ[nk], bket[1], mk[1], s.tk, Y.tk, tK,
                                              LOC_TJ[nb], bbra[1], mb[1])
                    if c9 == 0.0:
                        continue
                    sign = -1.0 if (Y.odd and LOC_N[nk] % 2) else 1.0
                    key = (mb, mk)
                    if key not in out.blocks:
                        out.blocks[key] = np.zeros((E.dim[mb], E.dim[mk]))
                    ob, ok = E.off[(mb, nb, bbra)], E.off[(mk, nk, bket)]
                    out.blocks[key][ob:ob + ym.shape[0], ok:ok + ym.shape[1]] += coef * c9 * sign * sv * ym


def identity_op(dims: dict) -> Op:
    return Op(0, 0, 0, False, {(q, q): np.eye(d) for q, d in dims.items()})


# ---------------------------------------------------------------------------
# Operator families of a block
#   ('H',)            block Hamiltonian (rank 0)
#   ('C', z)          b+_z for z in the block (rank 1/2)
#   ('S', w)          S_w = sum_{p,r,s in block} W_{w p r s} b+_p E_rs, w outside
#   ('A', tj, z, z')  [b+_z b+_z']^j           z <= z' in the block   (bare mode)
#   ('B', tj, z, z')  [b+_z b_z']^j            z <= z' in the block   (bare mode)
#   ('P', tj, w, w')  sum_{zz'} W_{z w z' w'} A^j_{zz'}   w <= w' outside (compl mode)
#   ('Q', tj, a, b)   sum_{rs} q^j_ab(r,s) B^j_rs         a <= b outside (compl mode)
#       q^0_ab(r,s) = 2 W_{abrs} - W_{rbas},  q^1_ab(r,s) = W_{rbas}
# Left and right blocks store the same families (creation-like orientation).
# ---------------------------------------------------------------------------
def qcoef(W, tj, a, b, r, s):
    if tj == 0:
        return 2.0 * W[a, b, r, s] - W[r, b, a, s]
    return W[r, b, a, s]


class Block:
    def __init__(self, side, bond, dims, orbs):
        self.side, self.bond, self.dims, self.orbs = side, bond, dict(dims), list(orbs)
        self.ops = {}


def _g(P, *orbs):
    g = 0
    for o in orbs:
        g ^= int(P.orb_irrep[o])
    return g


def get_A(Bk, P, tj, z, zp):
    if z <= zp:
        return Bk.ops.get(("A", tj, z, zp)), 1.0
    return Bk.ops.get(("A", tj, zp, z)), (-1.0) ** (tj // 2)


def get_B(Bk, P, tj, r, s):
    """B^j_rs from storage: B^j_sr = (-1)^j Tbar(B^j_rs)."""
    if r <= s:
        return Bk.ops.get(("B", tj, r, s))
    op = Bk.ops.get(("B", tj, s, r))
    return None if op is None else scale(adjoint(op), (-1.0) ** (tj // 2))


def get_P(Bk: Block, P: Problem, tj, w, wp) -> Op:
    """P^j_{w w'}(block): stored (compl mode) or summed from bare pairs."""
    g = _g(P, w, wp)
    if Bk.side == "L":
        mode = P.mode_left(Bk.bond)
    else:
        mode = P.mode_right(Bk.bond)
    if mode == "compl":
        if w <= wp:
            return Bk.ops[("P", tj, w, wp)]
        return scale(Bk.ops[("P", tj, wp, w)], (-1.0) ** (tj // 2))
    terms = []
    for z in Bk.orbs:
        for zp in Bk.orbs:
            c = P.W[z, w, zp, wp]
            if c == 0.0:
                continue
            op, f = get_A(Bk, P, tj, z, zp)
            if op is not None:
                terms.append((c * f, op))
    return lincomb(terms, tj, 2, g, False)


def get_Q(Bk: Block, P: Problem, tj, a, b) -> Op:
    g = _g(P, a, b)
    mode = P.mode_left(Bk.bond) if Bk.side == "L" else P.mode_right(Bk.bond)
    if mode == "compl":
        if a <= b:
            return Bk.ops[("Q", tj, a, b)]
        return scale(adjoint(Bk.ops[("Q", tj, b, a)]), (-1.0) ** (tj // 2))
    terms = []
    for r in Bk.orbs:
        for s in Bk.orbs:
            c = qcoef(P.W, tj, a, b, r, s)
            if c == 0.0:
                continue
            op = get_B(Bk, P, tj, r, s)
            if op is not None:
                terms.append((c, op))
    return lincomb(terms, tj, 0, g, False)


def cdag_combo(Bk: Block, P: Problem, coefs) -> Op:
    """sum_z coefs[z] b+_z (None if all zero)."""
    terms = [(c, Bk.ops[("C", z)]) for z, c in coefs.items() if c != 0.0]
    if not terms:
        return None
    z0 = next(z for z, c in coefs.items() if c != 0.0)
    return lincomb(terms, 1, 1, int(P.orb_irrep[z0]), True)


# ---------------------------------------------------------------------------
# Blocking: left block at bond k  (x)  site k  ->  enlarged left at bond k+1
# ---------------------------------------------------------------------------
def enlarge_left(P: Problem, X: Block, E: LeftEnl) -> Block:
    k = X.bond
    W = P.W
    gk = int(P.orb_irrep[k])
    orbs = X.orbs + [k]
    out = Block("L", k + 1, E.dim, orbs)
    comp = list(range(k + 1, P.L))
    Xops = X.ops

    def new(tk, dN, dG, odd):
        return Op(tk, dN, dG, odd, {})

    # C
    for x in X.orbs:
        o = new(1, 1, int(P.orb_irrep[x]), True)
        couple_left(o, Xops[("C", x)], SITE_I, E, 1.0)
        out.ops[("C", x)] = o
    o = new(1, 1, gk, True)
    couple_left(o, identity_op(X.dims), SITE_CDAG, E, 1.0)
    out.ops[("C", k)] = o
    Ik = identity_op(X.dims)

    # H
    o = new(0, 0, 0, False)
    couple_left(o, Xops[("H",)], SITE_I, E, 1.0)
    couple_left(o, Ik, site_h(W[k, k, k, k]), E, 1.0)
    t = new(0, 0, 0, False)
    couple_left(t, Xops[("S", k)], SITE_C, E, -SQ2)
    cx = cdag_combo(X, P, {x: W[x, k, k, k] for x in X.orbs})
    if cx is not None:
        couple_left(t, cx, SITE_E_C, E, -SQ2)
    Pkk = get_P(X, P, 0, k, k)
    couple_left(t, Pkk, SITE_AA0, E, -0.5)
    o = lincomb([(1.0, o), (1.0, plus_transpose(t))], 0, 0, 0, False)
    couple_left(o, get_Q(X, P, 0, k, k), SITE_B[0], E, 1.0)
    couple_left(o, get_Q(X, P, 2, k, k), SITE_B[2], E, SQ3)
    out.ops[("H",)] = o

    # S_y for y outside the enlarged block
    for y in comp:
        gy = int(P.orb_irrep[y])
        o = new(1, 1, gy, True)
        couple_left(o, Xops[("S", y)], SITE_I, E, 1.0)
        couple_left(o, get_Q(X, P, 0, k, y), SITE_CDAG, E, -1.0 / SQ2)
        couple_left(o, get_Q(X, P, 2, k, y), SITE_CDAG, E, -math.sqrt(1.5))
        couple_left(o, get_P(X, P, 0, y, k), SITE_C, E, 1.0 / SQ2)
        couple_left(o, get_P(X, P, 2, y, k), SITE_C, E, -math.sqrt(1.5))
        cs = cdag_combo(X, P, {s: W[k, y, k, s] for s in X.orbs})
        if cs is not None:
            couple_left(o, adjoint(cs), SITE_A0, E, 1.0 / SQ2)
        c0 = cdag_combo(X, P, {r: W[k, y, r, k] / SQ2 - SQ2 * W[r, y, k, k] for r in X.orbs})
        if c0 is not None:
            couple_left(o, c0, SITE_B[0], E, 1.0)
        c1 = cdag_combo(X, P, {r: W[k, y, r, k] for r in X.orbs})
        if c1 is not None:
            couple_left(o, c1, SITE_B[2], E, math.sqrt(1.5))
        couple_left(o, Ik, SITE_CDAG_E, E, W[k, y, k, k])
        out.ops[("S", y)] = o

    if P.mode_left(k + 1) == "bare":
        for x in orbs:
            for xp in orbs:
                if xp < x:
                    continue
                for tj in (0, 2):
                    g = _g(P, x, xp)
                    if not (x == xp and tj == 2):
                        o = new(tj, 2, g, False)
                        if xp < k:
                            couple_left(o, Xops[("A", tj, x, xp)], SITE_I, E, 1.0)
                        elif x < k:
                            couple_left(o, Xops[("C", x)], SITE_CDAG, E, 1.0)
                        else:
                            couple_left(o, Ik, SITE_A0, E, 1.0)
                        out.ops[("A", tj, x, xp)] = o
                    o = new(tj, 0, g, False)
                    if xp < k:
                        couple_left(o, Xops[("B", tj, x, xp)], SITE_I, E, 1.0)
                    elif x < k:
                        couple_left(o, Xops[("C", x)], SITE_C, E, 1.0)
                    else:
                        couple_left(o, Ik, SITE_B[tj], E, 1.0)
                    out.ops[("B", tj, x, xp)] = o
    else:
        for w in comp:
            for wp in comp:
                if wp < w:
                    continue
                g = _g(P, w, wp)
                for tj in (0, 2):
                    sg = (-1.0) ** (tj // 2)
                    if not (w == wp and tj == 2):
                        o = new(tj, 2, g, False)
                        couple_left(o, get_P(X, P, tj, w, wp), SITE_I, E, 1.0)
                        cz = cdag_combo(X, P, {z: W[z, w, k, wp] + sg * W[k, w, z, wp] for z in X.orbs})
                        if cz is not None:
                            couple_left(o, cz, SITE_CDAG, E, 1.0)
                        if tj == 0:
                            couple_left(o, Ik, SITE_A0, E, W[k, w, k, wp])
                        out.ops[("P", tj, w, wp)] = o
                    o = new(tj, 0, g, False)
                    couple_left(o, get_Q(X, P, tj, w, wp), SITE_I, E, 1.0)
                    cr = cdag_combo(X, P, {r: qcoef(W, tj, w, wp, r, k) for r in X.orbs})
                    if cr is not None:
                        couple_left(o, cr, SITE_C, E, 1.0)
                    cs = cdag_combo(X, P, {s: qcoef(W, tj, w, wp, k, s) for s in X.orbs})
                    if cs is not None:
                        couple_left(o, adjoint(cs), SITE_CDAG, E, sg)
                    couple_left(o, Ik, SITE_B[tj], E, qcoef(W, tj, w, wp, k, k))
                    out.ops[("Q", tj, w, wp)] = o
    return out


# ---------------------------------------------------------------------------
# Blocking: site k  (x)  right block at bond k+1  ->  enlarged right at bond k
# ---------------------------------------------------------------------------
def enlarge_right(P: Problem, Y: Block, E: RightEnl) -> Block:
    k = Y.bond - 1
    W = P.W
    gk = int(P.orb_irrep[k])
    orbs = [k] + Y.orbs
    out = Block("R", k, E.dim, orbs)
    comp = list(range(0, k))
    Yops = Y.ops
    Ik = identity_op(Y.dims)

    def new(tk, dN, dG, odd):
        return Op(tk, dN, dG, odd, {})

    for y in Y.orbs:
        o = new(1, 1, int(P.orb_irrep[y]), True)
        couple_right(o, SITE_I, Yops[("C", y)], E, 1.0)
        out.ops[("C", y)] = o
    o = new(1, 1, gk, True)
    couple_right(o, SITE_CDAG, Ik, E, 1.0)
    out.ops[("C", k)] = o

    # H
    o = new(0, 0, 0, False)
    couple_right(o, SITE_I, Yops[("H",)], E, 1.0)
    couple_right(o, site_h(W[k, k, k, k]), Ik, E, 1.0)
    t = new(0, 0, 0, False)
    cy = cdag_combo(Y, P, {y: W[k, y, k, k] for y in Y.orbs})
    if cy is not None:
        couple_right(t, SITE_CDAG_E, adjoint(cy), E, -SQ2)
    couple_right(t, SITE_CDAG, adjoint(Yops[("S", k)]), E, -SQ2)
    couple_right(t, SITE_A0, adjoint(get_P(Y, P, 0, k, k)), E, 0.5)
    o = lincomb([(1.0, o), (1.0, plus_transpose(t))], 0, 0, 0, False)
    couple_right(o, SITE_B[0], get_Q(Y, P, 0, k, k), E, 1.0)
    couple_right(o, SITE_B[2], get_Q(Y, P, 2, k, k), E, SQ3)
    out.ops[("H",)] = o

    # S_x = sum W_{p x r s} b+_p E_rs: the outside index x is the partner of
    # the creator p, so every coefficient below keeps x in the second slot
    # next to its partner (this matters only when (pq|rs) != (qp|rs))
    for x in comp:
        gx = int(P.orb_irrep[x])
        o = new(1, 1, gx, True)
        couple_right(o, SITE_I, Yops[("S", x)], E, 1.0)
        couple_right(o, SITE_CDAG, get_Q(Y, P, 0, k, x), E, -1.0 / SQ2)
        couple_right(o, SITE_CDAG, get_Q(Y, P, 2, k, x), E, math.sqrt(1.5))
        couple_right(o, SITE_C, get_P(Y, P, 0, x, k), E, 1.0 / SQ2)
        couple_right(o, SITE_C, get_P(Y, P, 2, x, k), E, math.sqrt(1.5))
        cs = cdag_combo(Y, P, {s: W[k, x, k, s] for s in Y.orbs})
        if cs is not None:
            couple_right(o, SITE_A0, adjoint(cs), E, 1.0 / SQ2)
        c0 = cdag_combo(Y, P, {r: W[k, x, r, k] / SQ2 - SQ2 * W[r, x, k, k] for r in Y.orbs})
        if c0 is not None:
            couple_right(o, SITE_B[0], c0, E, 1.0)
        c1 = cdag_combo(Y, P, {r: W[k, x, r, k] for r in Y.orbs})
        if c1 is not None:
            couple_right(o, SITE_B[2], c1, E, -math.sqrt(1.5))
        couple_right(o, SITE_CDAG_E, Ik, E, W[x, k, k, k])
        out.ops[("S", x)] = o

    if P.mode_right(k) == "bare":
        for y in orbs:
            for yp in orbs:
                if yp < y:
                    continue
                g = _g(P, y, yp)
                for tj in (0, 2):
                    if not (y == yp and tj == 2):
                        o = new(tj, 2, g, False)
                        if y > k:
                            couple_right(o, SITE_I, Yops[("A", tj, y, yp)], E, 1.0)
                        elif yp > k:
                            couple_right(o, SITE_CDAG, Yops[("C", yp)], E, 1.0)
                        else:
                            couple_right(o, SITE_A0, Ik, E, 1.0)
                        out.ops[("A", tj, y, yp)] = o
                    o = new(tj, 0, g, False)
                    if y > k:
                        couple_right(o, SITE_I, Yops[("B", tj, y, yp)], E, 1.0)
                    elif yp > k:
                        couple_right(o, SITE_CDAG, adjoint(Yops[("C", yp)]), E, 1.0)
                    else:
                        couple_right(o, SITE_B[tj], Ik, E, 1.0)
                    out.ops[("B", tj, y, yp)] = o
    else:
        for w in comp:
            for wp in comp:
                if wp < w:
                    continue
                g = _g(P, w, wp)
                for tj in (0, 2):
                    sg = (-1.0) ** (tj // 2)
                    if not (w == wp and tj == 2):
                        o = new(tj, 2, g, False)
                        couple_right(o, SITE_I, get_P(Y, P, tj, w, wp), E, 1.0)
                        cz = cdag_combo(Y, P, {z: W[k, w, z, wp] + sg * W[z, w, k, wp] for z in Y.orbs})
                        if cz is not None:
                            couple_right(o, SITE_CDAG, cz, E, 1.0)
                        if tj == 0:
                            couple_right(o, SITE_A0, Ik, E, W[k, w, k, wp])
                        out.ops[("P", tj, w, wp)] = o
                    o = new(tj, 0, g, False)
                    couple_right(o, SITE_I, get_Q(Y, P, tj, w, wp), E, 1.0)
                    cs = cdag_combo(Y, P, {s: qcoef(W, tj, w, wp, k, s) for s in Y.orbs})
                    if cs is not None:
                        couple_right(o, SITE_CDAG, adjoint(cs), E, 1.0)
                    cr = cdag_combo(Y, P, {r: qcoef(W, tj, w, wp, r, k) for r in Y.orbs})
                    if cr is not None:
                        couple_right(o, SITE_C, cr, E, sg)
                    couple_right(o, SITE_B[tj], Ik, E, qcoef(W, tj, w, wp, k, k))
                    out.ops[("Q", tj, w, wp)] = o
    return out


# ---------------------------------------------------------------------------
# Renormalisation (truncation of an enlarged block to a new bond basis)
# ---------------------------------------------------------------------------
def renorm_left(Xe: Block, U: dict, new_dims: dict) -> Block:
    """O' = U^T O U per sector pair; U[m] is (enlarged dim) x (kept dim)."""
    out = Block("L", Xe.bond, new_dims, Xe.orbs)
    for key, op in Xe.ops.items():
        o = Op(op.tk, op.dN, op.dG, op.odd, {})
        for (mb, mk), M in op.blocks.items():
            if mb in U and mk in U:
                o.blocks[(mb, mk)] = U[mb].T @ M @ U[mk]
        out.ops[key] = o
    return out


def renorm_right(Ye: Block, V: dict, new_dims: dict) -> Block:
    """O' = V O V^T per sector pair; V[m] is (kept dim) x (enlarged dim)."""
    out = Block("R", Ye.bond, new_dims, Ye.orbs)
    for key, op in Ye.ops.items():
        o = Op(op.tk, op.dN, op.dG, op.odd, {})
        for (mb, mk), M in op.blocks.items():
            if mb in V and mk in V:
                o.blocks[(mb, mk)] = V[mb] @ M @ V[mk].T
        out.ops[key] = o
    return out


# ---------------------------------------------------------------------------
# Two-site effective Hamiltonian
# ---------------------------------------------------------------------------
class Heff:
    """H_eff on psi = {m: (dimX[m], dimY[m]) matrix}, the singlet two-site basis."""

    def __init__(self, P: Problem, Xe: Block, Ye: Block, sectors):
        self.P, self.X, self.Y = P, Xe, Ye
        self.sectors = list(sectors)
        self.terms = []  # (coef, Xop, Yop, hc)
        X, Y = Xe.ops, Ye.ops
        Xorbs, Yorbs = Xe.orbs, Ye.orbs
        c = Xe.bond
        self.terms.append((1.0, X[("H",)], None, False))
        self.terms.append((1.0, None, Y[("H",)], False))
        for y in Yorbs:
            self.terms.append((-SQ2, X[("S", y)], adjoint(Y[("C", y)]), True))
        for x in Xorbs:
            self.terms.append((-SQ2, X[("C", x)], adjoint(Y[("S", x)]), True))
        if P.mode_left(c) == "bare":
            for x in Xorbs:
                for xp in Xorbs:
                    if xp < x:
                        continue
                    for tj in (0, 2):
                        if x < xp:
                            self.terms.append((math.sqrt(tj + 1), X[("A", tj, x, xp)],
                                               adjoint(Y[("P", tj, x, xp)]), True))
                            self.terms.append(((1.0, SQ3)[tj // 2], X[("B", tj, x, xp)],
                                               Y[("Q", tj, x, xp)], True))
                        else:
                            if tj == 0:
                                self.terms.append((0.5, X[("A", 0, x, x)], adjoint(Y[("P", 0, x, x)]), True))
                            self.terms.append(((1.0, SQ3)[tj // 2], X[("B", tj, x, x)],
                                               Y[("Q", tj, x, x)], False))
        else:
            for y in Yorbs:
                for yp in Yorbs:
                    if yp < y:
                        continue
                    for tj in (0, 2):
                        if y < yp:
                            self.terms.append((math.sqrt(tj + 1), X[("P", tj, y, yp)],
                                               adjoint(Y[("A", tj, y, yp)]), True))
                            self.terms.append(((1.0, SQ3)[tj // 2], X[("Q", tj, y, yp)],
                                               Y[("B", tj, y, yp)], True))
                        else:
                            if tj == 0:
                                self.terms.append((0.5, X[("P", 0, y, y)], adjoint(Y[("A", 0, y, y)]), True))
                            self.terms.append(((1.0, SQ3)[tj // 2], X[("Q", tj, y, y)],
                                               Y[("B", tj, y, y)], False))

    def _apply_term(self, out, psi, coef, Xo, Yo, transpose):
        secs = psi.keys()
        if Yo is None:  # X (x) 1, rank 0
            for (mb, mk), M in Xo.blocks.items():
                if mb in secs and mk in secs:
                    if transpose:
                        out[mk] += coef * M.T @ psi[mb]
                    else:
                        out[mb] += coef * M @ psi[mk]
            return
        if Xo is None:  # 1 (x) Y
            for (mb, mk), M in Yo.blocks.items():
                if mb in secs and mk in secs:
                    if transpose:
                        out[mk] += coef * psi[mb] @ M
                    else:
                        out[mb] += coef * psi[mk] @ M.T
            return
        tk = Xo.tk
        for (mb, mk), MX in Xo.blocks.items():
            if mb not in secs or mk not in secs:
                continue
            MY = Yo.blocks.get((mb, mk))
            if MY is None:
                continue
            cs = su2.product_coupling(mk[1], mk[1], 0, tk, tk, 0, mb[1], mb[1], 0)
            sign = -1.0 if (Yo.odd and mk[0] % 2) else 1.0
            f = coef * cs * sign
            if transpose:
                out[mk] += f * MX.T @ psi[mb] @ MY
            else:
                out[mb] += f * MX @ psi[mk] @ MY.T

    def apply(self, psi: dict) -> dict:
        out = {m: np.zeros_like(v) for m, v in psi.items()}
        for coef, Xo, Yo, hc in self.terms:
            self._apply_term(out, psi, coef, Xo, Yo, False)
            if hc:
                self._apply_term(out, psi, coef, Xo, Yo, True)
        return out

    def diagonal(self, shapes: dict) -> dict:
        out = {m: np.zeros(s) for m, s in shapes.items()}
        for coef, Xo, Yo, hc in self.terms:
            mult = 2.0 if hc else 1.0
            if Yo is None:
                for (mb, mk), M in Xo.blocks.items():
                    if mb == mk and mb in out:
                        out[mb] += mult * coef * np.diag(M)[:, None]
                continue
            if Xo is None:
                for (mb, mk), M in Yo.blocks.items():
                    if mb == mk and mb in out:
                        out[mb] += mult * coef * np.diag(M)[None, :]
                continue
            for (mb, mk), MX in Xo.blocks.items():
                if mb != mk or mb not in out:
                    continue
                MY = Yo.blocks.get((mb, mk))
                if MY is None:
                    continue
                cs = su2.product_coupling(mk[1], mk[1], 0, Xo.tk, Xo.tk, 0, mb[1], mb[1], 0)
                sign = -1.0 if (Yo.odd and mk[0] % 2) else 1.0
                out[mb] += mult * coef * cs * sign * np.outer(np.diag(MX), np.diag(MY))
        return out


def flatten(psi: dict, order) -> np.ndarray:
    return np.concatenate([psi[m].ravel() for m in order]) if order else np.zeros(0)


def unflatten(v: np.ndarray, shapes: dict, order) -> dict:
    out, o = {}, 0
    for m in order:
        n = shapes[m][0] * shapes[m][1]
        out[m] = v[o:o + n].reshape(shapes[m])
        o += n
    return out


def davidson(matvec, diag, x0, tol=1e-9, max_sub=32, max_iter=200):
    """Lowest eigenpair of a symmetric operator (Davidson 1975, diagonal preconditioner).

    Returns (theta, x, iterations, converged).
    """
    n = x0.size
    x = x0 / np.linalg.norm(x0)
    if n == 1:
        th = float(x @ matvec(x))
        return th, x, 1, True
    V = [x]
    AV = [matvec(x)]
    theta, conv, it = 0.0, False, 0
    for it in range(1, max_iter + 1):
        Vm = np.stack(V, axis=1)
        AVm = np.stack(AV, axis=1)
        Hs = Vm.T @ AVm
        Hs = 0.5 * (Hs + Hs.T)
        w, s = np.linalg.eigh(Hs)
        theta = float(w[0])
        x = Vm @ s[:, 0]
        ax = AVm @ s[:, 0]
        r = ax - theta * x
        if np.linalg.norm(r) <= tol:
            conv = True
            break
        den = theta - diag
        den = np.where(np.abs(den) < 1e-12, np.copysign(1e-12, den), den)
        t = r / den
        for _ in range(2):
            t = t - Vm @ (Vm.T @ t)
        nt = np.linalg.norm(t)
        if nt < 1e-14:
            t = r - Vm @ (Vm.T @ r)
            nt = np.linalg.norm(t)
            if nt < 1e-14:
                conv = True
                break
        t /= nt
        if len(V) >= max_sub:
            # restart with the current Ritz vector and the previous one
            x1 = x / np.linalg.norm(x)
            V = [x1]
            AV = [ax / np.linalg.norm(x)]
            t = t - x1 * (x1 @ t)
            t /= np.linalg.norm(t)
        V.append(t)
        AV.append(matvec(t))
    return theta, x / np.linalg.norm(x), it, conv


# ---------------------------------------------------------------------------
# MPS: left tensors U[i] (enlarged-left at bond i+1 -> bond i+1), right tensors
# V[i] (bond i -> enlarged-right at bond i), and the two-site centre.
# ---------------------------------------------------------------------------
@dataclass
class SweepStats:
    energies: list = field(default_factory=list)
    wdisc: list = field(default_factory=list)
    dav_iters: list = field(default_factory=list)


class DMRG:
    def __init__(self, P: Problem, D: int, seed: int = 7, dav_tol=1e-9, dav_max_sub=32, dav_max_iter=200):
        self.P = P
        self.seed = seed
        self.dav_tol, self.dav_max_sub, self.dav_max_iter = dav_tol, dav_max_sub, dav_max_iter
        self.caps = fci_caps(P)
        for k in range(P.L + 1):
            if not self.caps[k]:
                raise ValueError("target symmetry sector is empty")
        self.dims = [distribute(D, self.caps[k]) for k in range(P.L + 1)]
        self.Lblk = [None] * (P.L + 1)
        self.Rblk = [None] * (P.L + 1)
        self.U = [None] * P.L
        self.V = [None] * P.L
        self.center = None  # (i, psi dict) for the two-site object on sites i,i+1
        self.emin = math.inf
        self.stats = SweepStats()
        # noise (section "Convergence scheme"): bounded by 0.5 gamma w_disc of
        # the previous left- or right-sweep; passes counted from here
        self.n_pass = 0
        self.wd_prev = 0.0
        self.wd_pass = 0.0
        self.lower = []  # LowerState objects (excited-state solves)
        self._init_mps()

    # ----- initial state: random right-canonical tensors (paper: random noise)
    def _init_mps(self):
        P = self.P
        L = P.L
        # right tensors V[k], k = L-1 .. 1, for bond k
        for k in range(L - 1, 0, -1):
            E = RightEnl(P, k, self.dims[k + 1], keep=set(self.dims[k]))
            Vk = {}
            newd = {}
            for qi, m in enumerate(sorted(self.dims[k])):
                if m not in E.dim:
                    continue
                d, n = self.dims[k][m], E.dim[m]
                vals = _mps_random(self.seed, k, qi, d * n).reshape(d, n)
                # orthonormal rows (Gram-Schmidt via QR of the transpose)
                q, _ = np.linalg.qr(vals.T)
                r = min(d, n)
                Vk[m] = q[:, :r].T
                newd[m] = r
            self.V[k] = Vk
            self.dims[k] = newd
        E0 = LeftEnl(P, 1, self.dims[0], keep=set(self.dims[1]))
        psi = {}
        for qi, m in enumerate(sorted(self.dims[1])):
            if m not in E0.dim:
                continue
            d, n = E0.dim[m], self.dims[1][m]
            T0 = _mps_random(self.seed, 0, qi, d * n).reshape(d, n)
            psi[m] = T0  # enlarged-left at bond 1 x bond 1
        self._T0 = psi

    def build_boundaries(self):
        P = self.P
        L = P.L
        lb = Block("L", 0, {(0, 0, 0): 1}, [])
        lb.ops[("H",)] = zero_like(0, 0, 0, False)
        for y in range(L):
            lb.ops[("S", y)] = zero_like(1, 1, int(P.orb_irrep[y]), True)
        self.Lblk[0] = lb
        rb = Block("R", L, {(P.N, P.twoS, P.irrep): 1}, [])
        rb.ops[("H",)] = zero_like(0, 0, 0, False)
        for x in range(L):
            rb.ops[("S", x)] = zero_like(1, 1, int(P.orb_irrep[x]), True)
        self.Rblk[L] = rb
        for k in range(L - 1, 1, -1):
            E = RightEnl(P, k, self.Rblk[k + 1].dims, keep=set(self.dims[k]))
            Ye = enlarge_right(P, self.Rblk[k + 1], E)
            self.Rblk[k] = renorm_right(Ye, self.V[k], self.dims[k])
        # initial two-site object on sites 0,1 (bond 1): T0 (x) V[1]
        E = RightEnl(P, 1, self.dims[2], keep=set(self.dims[1]))
        self.center = (0, {m: self._T0[m] @ self.V[1][m] for m in self._T0 if m in self.V[1]})

    def build_blocks_at(self, i):
        """Left blocks at bonds 0..i from U[0..i-1] and right blocks at bonds
        L..i+2 from V[i+2..L-1] (for an MPS with its centre on (i, i+1))."""
        P = self.P
        L = P.L
        lb = Block("L", 0, {(0, 0, 0): 1}, [])
        lb.ops[("H",)] = zero_like(0, 0, 0, False)
        for y in range(L):
            lb.ops[("S", y)] = zero_like(1, 1, int(P.orb_irrep[y]), True)
        self.Lblk[0] = lb
        for c in range(1, i + 1):
            E = LeftEnl(P, c, self.Lblk[c - 1].dims, keep=set(self.dims[c]))
            self.Lblk[c] = renorm_left(enlarge_left(P, self.Lblk[c - 1], E), self.U[c - 1], self.dims[c])
        rb = Block("R", L, {(P.N, P.twoS, P.irrep): 1}, [])
        rb.ops[("H",)] = zero_like(0, 0, 0, False)
        for x in range(L):
            rb.ops[("S", x)] = zero_like(1, 1, int(P.orb_irrep[x]), True)
        self.Rblk[L] = rb
        for k in range(L - 1, i + 1, -1):
            E = RightEnl(P, k, self.Rblk[k + 1].dims, keep=set(self.dims[k]))
            self.Rblk[k] = renorm_right(enlarge_right(P, self.Rblk[k + 1], E), self.V[k], self.dims[k])

    # ----- one micro-iteration
    def enlarged(self, i):
        P = self.P
        c = i + 1
        Lk, Rk = self.Lblk[i], self.Rblk[i + 2]
        El0 = LeftEnl(P, c, Lk.dims)
        Er0 = RightEnl(P, c, Rk.dims)
        keep = set(El0.dim) & set(Er0.dim)
        El = LeftEnl(P, c, Lk.dims, keep=keep)
        Er = RightEnl(P, c, Rk.dims, keep=keep)
        Xe = enlarge_left(P, Lk, El)
        Ye = enlarge_right(P, Rk, Er)
        return El, Er, Xe, Ye, sorted(keep)

    def micro(self, i, D, direction, do_svd=True, noise=0.0):
        P = self.P
        El, Er, Xe, Ye, secs = self.enlarged(i)
        H = Heff(P, Xe, Ye, secs)
        shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
        ci, guess = self.center
        assert ci == i
        x0 = flatten({m: guess.get(m, np.zeros(shapes[m])) for m in secs}, secs)
        if np.linalg.norm(x0) == 0:
            x0 = np.ones_like(x0)
        dg = flatten(H.diagonal(shapes), secs)
        phis = [(w.eta, flatten(project_lower(P, self, w, i, El, Er, secs), secs)) for w in self.lower]
        for eta, f in phis:
            dg = dg + eta * f * f

        def mv(v):
            y = flatten(H.apply(unflatten(v, shapes, secs)), secs)
            for eta, f in phis:
                y = y + eta * (f @ v) * f
            return y
        th, x, its, conv = davidson(mv, dg, x0, self.dav_tol, self.dav_max_sub, self.dav_max_iter)
        e = th + P.e_const
        self.emin = min(self.emin, e)
        self.stats.energies.append(e)
        self.stats.dav_iters.append(its)
        if not do_svd:
            self.center = (i, unflatten(x, shapes, secs))
            return e
        if noise > 0.0 and self.wd_prev > 0.0:
            # uniform noise of magnitude <= 0.5 gamma w_disc(previous pass),
            # added just before the decomposition (section "Convergence scheme");
            # the eigenvector's arbitrary sign is fixed first (<x, u> >= 0) so
            # that the noisy object does not depend on it
            u = noise_values(self.seed, self.n_pass, i, len(x))
            if x @ u < 0:
                x = -x
            x = x + 0.5 * noise * self.wd_prev * u
        psi = unflatten(x, shapes, secs)
        U, s, Vt, kept, wd = svd_truncate(psi, D)
        self.stats.wdisc.append(wd)
        self.wd_pass = max(self.wd_pass, wd)
        c = i + 1
        if direction == "right":
            self.U[i] = U
            self.dims[c] = kept
            self.Lblk[c] = renorm_left(Xe, U, kept)
            C = {m: s[m][:, None] * Vt[m] for m in kept}
            self.center = (i + 1, move_center_right(P, C, self.V[i + 2], c, kept, self.dims[c + 1]))
        else:
            self.V[i + 1] = Vt
            self.dims[c] = kept
            self.Rblk[c] = renorm_right(Ye, Vt, kept)
            C = {m: U[m] * s[m][None, :] for m in kept}
            self.center = (i - 1, move_center_left(P, C, self.U[i - 1], c, kept, self.dims[c - 1]))
        return e

    def push_lower(self, other, eta):
        """Project the state of `other` (a DMRG of the same problem, centre at
        the left end) out of this one's solves with weight eta."""
        self.lower.append(LowerState(other, eta))

    def sweep(self, D, noise=0.0):
        """One macro-iteration: right pass i = 0..L-2, left pass i = L-2..0.

        The turning steps are not split: at i = L-2 of the right pass and at
        i = 0 of the left pass the optimised two-site object is kept as the
        guess for the first step of the next pass.
        """
        L = self.P.L
        e0 = len(self.stats.energies)
        for i in range(0, L - 1):
            self.micro(i, D, "right", do_svd=(i < L - 2), noise=noise)
        self._end_pass()
        for i in range(L - 2, -1, -1):
            self.micro(i, D, "left", do_svd=(i > 0), noise=noise)
        self._end_pass()
        return min(self.stats.energies[e0:])

    def _end_pass(self):
        self.wd_prev, self.wd_pass = self.wd_pass, 0.0
        self.n_pass += 1

    def solve(self, schedule):
        """schedule: list of (D, e_conv, max_sweeps[, noise])."""
        if self.Rblk[2] is None:
            self.build_boundaries()
        e_prev = math.inf
        for ins in schedule:
            D, e_conv, nmax = ins[:3]
            noise = ins[3] if len(ins) > 3 else 0.0
            for _ in range(nmax):
                e = self.sweep(D, noise)
                if abs(e - e_prev) < e_conv:
                    e_prev = e
                    break
                e_prev = e
        return self.emin

    # two-site wavefunction as (sectors, shapes, flat vector) at the current centre
    def current_psi(self):
        return self.center


# ---------------------------------------------------------------------------
# Excited states by projection (section "CheMPS2 library", the DMRG object):
# after a state Psi_k is found it is pushed back with a weight eta_k > 0 and
# the next solve uses H_m = H_0 + sum_k eta_k |Psi_k><Psi_k|.  On the current
# two-site space the extra term is sum_k eta_k |phi_k><phi_k| with
# phi_k = P_i Psi_k the projection of Psi_k onto that space.  Here Psi_k's
# centre is first carried along the chain by exact decompositions (nothing
# truncated), so that its two-site object psi_k(i) at every step is at hand
# in its own left- and right-normalised bases; then
#   phi_k(i) = (OL(i) (x) 1 (x) 1 (x) OR(i+2)) psi_k(i),
# OL / OR the overlaps between the current and Psi_k's normalised left /
# right block states, built afresh from the chain ends at every step.
# ---------------------------------------------------------------------------
class LowerState:
    def __init__(self, dm, eta):
        P = dm.P
        i, psi = dm.center
        if i != 0:
            raise ValueError("push a lower state when its centre is at the left end")
        self.eta = float(eta)
        nrm = math.sqrt(sum(float(np.sum(x * x)) for x in psi.values()))
        self.dimsR = [dict(d) for d in dm.dims]        # right-normalised bases
        self.V = [None if v is None else {m: x.copy() for m, x in v.items()} for v in dm.V]
        self.dimsL = [dict(dm.dims[0])] + [None] * P.L  # left-normalised bases
        self.U = [None] * P.L
        self.psi = [None] * (P.L - 1)
        cur = {m: x / nrm for m, x in psi.items()}
        for j in range(P.L - 1):
            self.psi[j] = cur
            if j == P.L - 2:
                break
            U, s, Vt, kept, _ = svd_truncate(cur, 10 ** 9)
            self.U[j] = U
            self.dimsL[j + 1] = kept
            C = {m: s[m][:, None] * Vt[m] for m in kept}
            cur = move_center_right(P, C, self.V[j + 2], j + 1, kept, self.dimsR[j + 2])


def overlap_left(P, U_cur, dims_cur, U_k, dims_k, i):
    """<current left states at bond i | Psi_k's left-normalised states>."""
    O = {s: np.ones((1, 1)) for s in dims_cur[0]}
    for c in range(i):
        Ec, Ek = LeftEnl(P, c + 1, dims_cur[c]), LeftEnl(P, c + 1, dims_k[c])
        new = {}
        for m, Uc in U_cur[c].items():
            if m not in U_k[c] or m not in Ec.pieces:
                continue
            acc = np.zeros((Uc.shape[1], U_k[c][m].shape[1]))
            for (a, n) in Ec.pieces[m]:
                if a not in O or (m, a, n) not in Ek.off:
                    continue
                oc, ok = Ec.off[(m, a, n)], Ek.off[(m, a, n)]
                acc += Uc[oc:oc + dims_cur[c][a]].T @ O[a] @ U_k[c][m][ok:ok + dims_k[c][a]]
            new[m] = acc
        O = new
    return O


def overlap_right(P, V_cur, dims_cur, V_k, dims_k, b0):
    """<current right states at bond b0 | Psi_k's right-normalised states>."""
    O = {s: np.ones((1, 1)) for s in dims_cur[P.L]}
    for c in range(P.L - 1, b0 - 1, -1):
        Ec, Ek = RightEnl(P, c, dims_cur[c + 1]), RightEnl(P, c, dims_k[c + 1])
        new = {}
        for m, Vc in V_cur[c].items():
            if m not in V_k[c] or m not in Ec.pieces:
                continue
            acc = np.zeros((Vc.shape[0], V_k[c][m].shape[0]))
            for (n, b) in Ec.pieces[m]:
                if b not in O or (m, n, b) not in Ek.off:
                    continue
                oc, ok = Ec.off[(m, n, b)], Ek.off[(m, n, b)]
                acc += Vc[:, oc:oc + dims_cur[c + 1][b]] @ O[b] @ V_k[c][m][:, ok:ok + dims_k[c + 1][b]].T
            new[m] = acc
        O = new
    return O


def project_lower(P, dm, w: LowerState, i, El, Er, secs):
    """phi = P_i Psi_k on the current two-site space of step i."""
    OL = overlap_left(P, dm.U, dm.dims, w.U, w.dimsL, i)
    OR = overlap_right(P, dm.V, dm.dims, w.V, w.dimsR, i + 2)
    Elk, Erk = LeftEnl(P, i + 1, w.dimsL[i]), RightEnl(P, i + 1, w.dimsR[i + 2])
    out = {}
    for m in secs:
        phi = np.zeros((El.dim[m], Er.dim[m]))
        pk = w.psi[i].get(m)
        if pk is not None and m in Elk.pieces and m in Erk.pieces:
            for (a, n1) in El.pieces[m]:
                if a not in OL or (m, a, n1) not in Elk.off:
                    continue
                rc, rk = El.off[(m, a, n1)], Elk.off[(m, a, n1)]
                rows = OL[a] @ pk[rk:rk + w.dimsL[i][a]]
                for (n2, b) in Er.pieces[m]:
                    if b not in OR or (m, n2, b) not in Erk.off:
                        continue
                    cc, ck = Er.off[(m, n2, b)], Erk.off[(m, n2, b)]
                    phi[rc:rc + dm.dims[i][a], cc:cc + dm.dims[i + 2][b]] += (
                        rows[:, ck:ck + w.dimsR[i + 2][b]] @ OR[b].T)
        out[m] = phi
    return out


NOISE_STREAM = 0x4E4F << 40


def random_mps_at(P: Problem, D: int, seed: int, i: int) -> "DMRG":
    """A random MPS with its two-site centre on sites (i, i+1): the initial
    right-normalised tensors V[i+2..L-1] of DMRG(P, D, seed), random
    left-normalised tensors U[0..i-1] (orthonormal columns from the QR of
    counter-generated entries) and a counter-generated two-site object.  No
    blocks are built (build_blocks_at does that).  A deterministic input for
    parity checks at a chosen step without any optimisation."""
    dm = DMRG(P, D, seed=seed)
    for c in range(i):
        E = LeftEnl(P, c + 1, dm.dims[c], keep=set(dm.dims[c + 1]))
        U, newd = {}, {}
        for qi, m in enumerate(sorted(dm.dims[c + 1])):
            if m not in E.dim:
                continue
            rows, k = E.dim[m], dm.dims[c + 1][m]
            q, _ = np.linalg.qr(_mps_random(seed, (1 << 12) | c, qi, rows * k).reshape(rows, k))
            r = min(rows, k)
            U[m] = q[:, :r]
            newd[m] = r
        dm.U[c] = U
        dm.dims[c + 1] = newd
    El = LeftEnl(P, i + 1, dm.dims[i])
    Er = RightEnl(P, i + 1, dm.dims[i + 2])
    psi = {}
    for qi, m in enumerate(sorted(set(El.dim) & set(Er.dim))):
        psi[m] = _mps_random(seed, (1 << 13) | i, qi, El.dim[m] * Er.dim[m]).reshape(El.dim[m], Er.dim[m])
    dm.center = (i, psi)
    return dm


def noise_values(seed, n_pass, i, n):
    """The noise draws of step i of pass n_pass: uniform in [-1, 1), counter-based."""
    from synth.integrals import uniform_pm1_array
    return uniform_pm1_array(seed, NOISE_STREAM | (n_pass << 16) | i, n)


def _mps_random(seed, site, sector_index, n):
    from synth.integrals import uniform_pm1_array
    return uniform_pm1_array(seed, (site << 20) | sector_index, n)


def svd_truncate(psi: dict, D: int):
    """SVD per (j_M, N_M, I_M) sector; keep the D largest kappa = s/sqrt(2j_M+1).

    Returns U, s, Vt (truncated, per sector), kept dims, discarded weight
    w = sum_discarded s^2 (= sum over discarded multiplets of (2j+1) kappa^2).
    """
    Us, Ss, Vs = {}, {}, {}
    cand = []
    for qi, m in enumerate(sorted(psi)):
        u, s, vt = np.linalg.svd(psi[m], full_matrices=False)
        # sign convention: the largest-magnitude entry of each left singular
        # vector (lowest row among ties) is positive; the right vector follows
        for a in range(u.shape[1]):
            if u[np.argmax(np.abs(u[:, a])), a] < 0:
                u[:, a] = -u[:, a]
                vt[a, :] = -vt[a, :]
        Us[m], Ss[m], Vs[m] = u, s, vt
        for a, sv in enumerate(s):
            cand.append((-sv / math.sqrt(m[1] + 1), qi, a, m))
    cand.sort(key=lambda t: (t[0], t[1], t[2]))
    keep = cand[:D]
    norm2 = sum(float(np.sum(Ss[m] ** 2)) for m in Ss)
    kept = {}
    for _, _, a, m in keep:
        kept[m] = kept.get(m, 0) + 1
    wd = sum(float(Ss[m][a] ** 2) for (_, _, a, m) in cand[D:]) / max(norm2, 1e-300)
    kept = dict(sorted(kept.items()))
    U = {m: Us[m][:, :kept[m]] for m in kept}
    s = {m: Ss[m][:kept[m]] for m in kept}
    Vt = {m: Vs[m][:kept[m], :] for m in kept}
    return U, s, Vt, kept, wd


def recouple_singlet(tja, ts, tjb):
    """<[a (x) [s (x) b]^{ja}]^0 | [[a (x) s]^{jb} (x) b]^0>, explicit CG sum."""
    tot = 0.0
    for tmu in range(-tja, tja + 1, 2):
        c1 = su2.cg(tja, tmu, tja, -tmu, 0, 0)
        for tsig in range(-ts, ts + 1, 2):
            tbeta = -tmu - tsig
            if abs(tbeta) > tjb:
                continue
            c2 = su2.cg(ts, tsig, tjb, tbeta, tja, -tmu)
            tnu = tmu + tsig
            c3 = su2.cg(tjb, tnu, tjb, tbeta, 0, 0)
            c4 = su2.cg(tja, tmu, ts, tsig, tjb, tnu)
            tot += c1 * c2 * c3 * c4
    return tot


def move_center_right(P: Problem, C: dict, Vnext: dict, c: int, dims_c: dict, dims_c1: dict) -> dict:
    """New two-site object on sites (c, c+1) from C[a] (a at bond c, right-enlarged
    columns (n, b) at bond c) and the right tensor Vnext at bond c+1."""
    Er = RightEnl(P, c, dims_c1)
    El_new = LeftEnl(P, c + 1, dims_c)
    out = {}
    for a, Ca in C.items():
        if a not in Er.pieces:
            continue
        for (n, b) in Er.pieces[a]:
            # piece (n at site c, b at bond c+1): b is the middle sector of the new object
            if b not in Vnext or (b, a, n) not in El_new.off:
                continue
            off = Er.off[(a, n, b)]
            blk = Ca[:, off:off + dims_c1[b]] @ Vnext[b]
            r = recouple_singlet(a[1], LOC_TJ[n], b[1])
            if b not in out:
                out[b] = np.zeros((El_new.dim[b], Vnext[b].shape[1]))
            ro = El_new.off[(b, a, n)]
            out[b][ro:ro + blk.shape[0], :] += r * blk
    return out


def recouple_singlet_left(tja, ts, tjb):
    """<[[a (x) s]^{jb} (x) b]^0 | [a (x) [s (x) b]^{ja}]^0> (same overlap)."""
    return recouple_singlet(tja, ts, tjb)


def move_center_left(P: Problem, C: dict, Uprev: dict, c: int, dims_c: dict, dims_cm1: dict) -> dict:
    """New two-site object on sites (c-2, c-1) from C[b] (left-enlarged rows
    (a, n) at bond c, columns = bond-c sector b) and the left tensor Uprev."""
    El = LeftEnl(P, c, dims_cm1)
    Er_new = RightEnl(P, c - 1, dims_c)
    out = {}
    for b, Cb in C.items():
        if b not in El.pieces:
            continue
        for (a, n) in El.pieces[b]:
            # piece (a at bond c-1, n at site c-1): a is the new middle sector
            if a not in Uprev or (a, n, b) not in Er_new.off:
                continue
            off = El.off[(b, a, n)]
            blk = Uprev[a] @ Cb[off:off + dims_cm1[a], :]
            r = recouple_singlet(a[1], LOC_TJ[n], b[1])
            if a not in out:
                out[a] = np.zeros((Uprev[a].shape[0], Er_new.dim[a]))
            co = Er_new.off[(a, n, b)]
            out[a][:, co:co + blk.shape[1]] += r * blk
    return out


# ---------------------------------------------------------------------------
# MPS blob (the exchange format declared in the C ABI header), written from the
# oracle's state so that the GPU path can be run on the same tensors.
# ---------------------------------------------------------------------------
MPS_MAGIC = 0x3154535053414453


def export_blob(dm: DMRG) -> bytes:
    import struct
    P = dm.P
    i, psi = dm.center
    out = bytearray()

    def put(*vals):
        for v in vals:
            out.extend(struct.pack("<q", int(v)))

    def putm(a):
        out.extend(np.ascontiguousarray(a, dtype="<f8").tobytes())

    put(MPS_MAGIC, P.L, P.N, P.twoS, P.irrep, i)
    for k in range(P.L + 1):
        d = dm.dims[k]
        put(len(d))
        for q in sorted(d):
            put(q[0], q[1], q[2], d[q])
    for k in range(i):
        for m in sorted(dm.dims[k + 1]):
            putm(dm.U[k][m])
    for k in range(i + 2, P.L):
        for m in sorted(dm.dims[k]):
            putm(dm.V[k][m])
    El = LeftEnl(P, i + 1, dm.dims[i])
    Er = RightEnl(P, i + 1, dm.dims[i + 2])
    for m in sorted(El.dim):
        if m in Er.dim:
            putm(psi.get(m, np.zeros((El.dim[m], Er.dim[m]))))
    return bytes(out)
