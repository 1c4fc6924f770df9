"""Pins for the oracle's spin-adapted DMRG.

* sigma = P^T H P x from an explicit Fock-space expansion (all term families,
  both pair modes, several spins and point groups, truncated bonds);
* renormalised and complementary operators equal explicit <alpha|O|beta>;
* sector tables against closed-form counts;
* energies: exact at the FCI bond dimension, variational below it.
"""
import math

import numpy as np
import pytest

from oracle import sadmrg as sd
from oracle import su2
from oracle.explicit import Expansion, Fock
from oracle.fci import fci_solve
from synth.integrals import fourfold_eri, make_integrals

CASES = [(4, 4, 2, "C1", 0, 16), (5, 5, 1, "C2v", 1, 16), (6, 6, 0, "C1", 0, 6), (6, 5, 3, "C2", 1, 8),
         (6, 6, 4, "D2h", 0, 10), (6, 7, 1, "C2v", 3, 7)]


def _setup(L, N, twoS, group, irrep, D, seed=11, four=False):
    I = make_integrals(L, group, seed)
    if four:  # integrals with only (pq|rs) = (rs|pq) = (qp|sr)
        I.eri = fourfold_eri(I, seed + 100)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    return I, P, dm


@pytest.mark.parametrize("four", [False, True])
@pytest.mark.parametrize("case", CASES)
def test_sigma_equals_projected_hamiltonian(case, four):
    """Also with integrals that keep only the symmetry of a real two-body
    operator: every blocking formula must read each integral with the
    creator-annihilator pairing of the term it builds."""
    if four and case[0] > 5 and case[3] == "C1" and case[2] == 0:
        pytest.skip("covered by the other four-fold cases")
    I, P, dm = _setup(*case, four=four)
    L, D = P.L, case[-1]
    F = Fock(L)
    H = F.hamiltonian(I.h, I.eri)  # unfolded integrals: also checks the folding
    ex = Expansion(dm, F)
    for i in range(L - 1):
        El, Er, Xe, Ye, secs = dm.enlarged(i)
        He = sd.Heff(P, Xe, Ye, secs)
        shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
        rng = np.random.default_rng(i)
        psi = {m: rng.normal(size=shapes[m]) for m in secs}
        sig = He.apply(psi)
        B = np.concatenate([v for v in ex.two_site_basis(i, El, Er, secs, ex.left_states(i),
                                                         ex.right_states(i + 2)).values()], axis=0)
        assert np.abs(B @ B.T - np.eye(len(B))).max() < 1e-12  # orthonormal two-site basis
        x = np.concatenate([psi[m].ravel() for m in secs])
        ref = B @ (H @ (B.T @ x).reshape(F.dim, P.twoS + 1)).ravel()
        got = np.concatenate([sig[m].ravel() for m in secs])
        assert np.abs(got - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())
        dg = He.diagonal(shapes)
        dref = np.array([b @ (H @ b.reshape(F.dim, P.twoS + 1)).ravel() for b in B])
        assert np.abs(np.concatenate([dg[m].ravel() for m in secs]) - dref).max() < 1e-11
        if i < L - 2:
            dm.micro(i, D, "right")


def _explicit_family(F, P, key, orbs):
    """Top (q = k) component of a family operator as an explicit Fock matrix."""
    W = P.W
    cd = F.cdag

    def b(p, tq):  # b_{p,q} = (-1)^(1/2-q) a_{p,-q}
        sg = 1 if tq == 1 else 0  # a_{p,-q}: -q = -1/2 -> down(1) when q=+1/2
        return (-1.0 if tq == -1 else 1.0) * cd[p, sg].T

    def bd(p, tq):
        return cd[p, 0] if tq == 1 else cd[p, 1]

    def pair(f1, f2, p1, p2, tj):
        return sum(su2.cg(1, q1, 1, tj - q1, tj, tj) * (f1(p1, q1) @ f2(p2, tj - q1))
                   for q1 in (-1, 1) if abs(tj - q1) <= 1)

    fam = key[0]
    if fam == "H":
        Hm = 0
        for p in orbs:
            for q in orbs:
                for r in orbs:
                    for s in orbs:
                        if W[p, q, r, s] != 0.0:
                            t = F.E[p, q] @ F.E[r, s]
                            if q == r:
                                t = t - F.E[p, s]
                            Hm = Hm + 0.5 * W[p, q, r, s] * t
        return Hm
    if fam == "C":
        return bd(key[1], 1)
    if fam == "S":
        y = key[1]
        # the creator p is the partner of the outside annihilator y
        return sum(W[p, y, r, s] * (bd(p, 1) @ F.E[r, s]) for p in orbs for r in orbs for s in orbs
                   if W[p, y, r, s] != 0.0)
    if fam == "A":
        return pair(bd, bd, key[2], key[3], key[1])
    if fam == "B":
        return pair(bd, b, key[2], key[3], key[1])
    if fam == "P":
        tj, w, wp = key[1:]
        return sum(W[z, w, zp, wp] * pair(bd, bd, z, zp, tj) for z in orbs for zp in orbs if W[z, w, zp, wp] != 0.0)
    if fam == "Q":
        tj, a, bb = key[1:]
        return sum(sd.qcoef(W, tj, a, bb, r, s) * pair(bd, b, r, s, tj) for r in orbs for s in orbs
                   if sd.qcoef(W, tj, a, bb, r, s) != 0.0)
    raise KeyError(key)


@pytest.mark.parametrize("four", [False, True])
@pytest.mark.parametrize("case", [(6, 6, 2, "C1", 0, 8), (6, 5, 1, "C2", 1, 6)])
def test_renormalised_operators_equal_explicit(case, four):
    I, P, dm = _setup(*case, four=four)
    L, D = P.L, case[-1]
    F = Fock(L)
    ex = Expansion(dm, F)
    for i in range(L - 2):
        dm.micro(i, D, "right")
    for k in (2, 3, 4):
        blk = dm.Lblk[k]
        st = ex.left_states(k)
        for key, op in blk.ops.items():
            M = _explicit_family(F, P, key, blk.orbs)
            for (bra, ket), red in op.blocks.items():
                tk = op.tk
                tmp = bra[1] if bra[1] >= 0 else 0
                tm = tmp - tk
                if abs(tm) > ket[1]:
                    tm = ket[1]
                    tmp = tm + tk
                c = su2.cg(ket[1], tm, tk, tk, bra[1], tmp)
                if abs(c) < 1e-9:
                    continue
                Vb = st[bra][:, (tmp + bra[1]) // 2, :]
                Vk = st[ket][:, (tm + ket[1]) // 2, :]
                got = Vb @ (M @ Vk.T) if not np.isscalar(M) else 0 * red
                assert np.allclose(got, c * red, atol=1e-10), (k, key, bra, ket)
    # right blocks (orbitals to the right plus the ghost spin)
    dm2 = _setup(*case, four=four)[2]
    for k in (3, 4):
        blk = dm2.Rblk[k]
        st = ex.__class__(dm2, F).right_states(k)
        for key, op in blk.ops.items():
            M = _explicit_family(F, P, key, blk.orbs)
            for (bra, ket), red in op.blocks.items():
                tk = op.tk
                tmp = bra[1]
                tm = tmp - tk
                if abs(tm) > ket[1]:
                    tm = ket[1]
                    tmp = tm + tk
                c = su2.cg(ket[1], tm, tk, tk, bra[1], tmp)
                if abs(c) < 1e-9:
                    continue
                Vb = st[bra][:, (tmp + bra[1]) // 2]  # (d, fock, ghost)
                Vk = st[ket][:, (tm + ket[1]) // 2]
                MVk = np.stack([M @ Vk[r].reshape(F.dim, -1) for r in range(Vk.shape[0])])
                got = np.einsum("afg,bfg->ab", Vb, MVk)
                assert np.allclose(got, c * red, atol=1e-10), (k, key, bra, ket)


def test_sector_tables_config1():
    I = make_integrals(8, "C1", 1001)
    P = sd.Problem(I.h, I.eri, 8, 0, 0, I.orb_irrep)
    rm = sd.right_multiplicities(P)
    # number of N=8, S=0 spin-adapted configurations of 8 orbitals (Weyl):
    # dim(M=0) - dim(M=1) = C(8,4)^2 - C(8,5) C(8,3) = 1764
    assert rm[0][(0, 0, 0)] == 1764
    caps = sd.fci_caps(P)
    assert [sum(c.values()) for c in caps] == [1, 3, 10, 35, 126, 35, 10, 3, 1]


def test_distribute_respects_caps_and_total():
    caps = {(0, 0, 0): 2, (1, 1, 0): 50, (2, 0, 0): 7, (2, 2, 0): 100}
    d = sd.distribute(60, caps)
    assert sum(d.values()) == 60 and all(d[q] <= caps[q] for q in d)
    assert d[(0, 0, 0)] == 2 and d[(2, 0, 0)] == 7


def test_svd_truncation_normalisation():
    rng = np.random.default_rng(2)
    psi = {(4, 0, 0): rng.normal(size=(5, 7)), (4, 2, 0): rng.normal(size=(3, 4)), (5, 1, 1): rng.normal(size=(6, 2))}
    nrm = math.sqrt(sum(np.sum(v ** 2) for v in psi.values()))
    psi = {m: v / nrm for m, v in psi.items()}
    U, s, Vt, kept, wd = sd.svd_truncate(psi, 100)
    assert wd < 1e-14 and abs(sum(np.sum(x ** 2) for x in s.values()) - 1) < 1e-12
    for m in psi:
        assert np.allclose(U[m] @ np.diag(s[m]) @ Vt[m], psi[m])
        assert np.allclose(U[m].T @ U[m], np.eye(kept[m]))
    U, s, Vt, kept, wd = sd.svd_truncate(psi, 4)
    assert sum(kept.values()) == 4
    kap = sorted([x / math.sqrt(m[1] + 1) for m in s for x in s[m]], reverse=True)
    allk = sorted([x / math.sqrt(m[1] + 1) for m in psi for x in np.linalg.svd(psi[m], compute_uv=False)],
                  reverse=True)
    assert np.allclose(kap, allk[:4])
    assert abs(wd - (1 - sum(np.sum(x ** 2) for x in s.values()))) < 1e-12


def test_number_operator_invariant_on_bare_blocks():
    # sum_k E_kk = -sqrt2 sum_k B^0_kk equals N_a on every sector of a left block
    I, P, dm = _setup(6, 6, 0, "C1", 0, 8)
    for i in range(3):
        dm.micro(i, 8, "right")
    blk = dm.Lblk[3]
    assert P.mode_left(3) == "bare"
    tot = {}
    for k in blk.orbs:
        for (bra, ket), m in blk.ops[("B", 0, k, k)].blocks.items():
            tot[(bra, ket)] = tot.get((bra, ket), 0) - math.sqrt(2) * m
    for (bra, ket), m in tot.items():
        assert bra == ket
        assert np.allclose(m, bra[0] * np.eye(m.shape[0]), atol=1e-12)


def test_dmrg_config1_exact_at_fci_bond_dimension():
    I = make_integrals(8, "C1", 1001)
    efci = fci_solve(I.h, I.eri, 8, 0)[0][0]
    P = sd.Problem(I.h, I.eri, 8, 0, 0, I.orb_irrep)
    dm = sd.DMRG(P, 128, seed=7)
    e = dm.solve([(128, 1e-10, 3)])
    assert abs(e - efci) < 1e-10


@pytest.mark.parametrize("N,twoS,group,irrep", [(6, 2, "C1", 0), (5, 1, "C2v", 1), (6, 0, "D2h", 0)])
def test_dmrg_spin_and_symmetry_targets_exact(N, twoS, group, irrep):
    I = make_integrals(6, group, 21)
    efci = fci_solve(I.h, I.eri, N, twoS, irrep, I.orb_irrep)[0][0]
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, 64, seed=5)
    assert abs(dm.solve([(64, 1e-11, 3)]) - efci) < 1e-10


def test_dmrg_variational_and_monotone_in_D():
    I = make_integrals(8, "C1", 1001)
    efci = fci_solve(I.h, I.eri, 8, 0)[0][0]
    es = []
    for D in (4, 8, 16):
        P = sd.Problem(I.h, I.eri, 8, 0, 0, I.orb_irrep)
        dm = sd.DMRG(P, D, seed=7)
        dm.solve([(D, 1e-9, 3)])
        es.append(dm.stats.energies[-1])
    assert all(e >= efci - 1e-10 for e in es)
    assert es[0] >= es[1] - 1e-9 >= es[2] - 2e-9
    assert es[0] > efci + 1e-6


def test_noise_enters_after_the_first_pass_and_is_bounded():
    """Noise is 0.5 gamma w_disc(previous pass) times uniform draws: the first
    pass (no previous pass) equals the noiseless run; later passes differ but
    stay variational above FCI."""
    L, N, D = 8, 8, 12
    I = make_integrals(L, "C1", 1001)
    P = sd.Problem(I.h, I.eri, N, 0, 0, I.orb_irrep)
    e_fci = fci_solve(I.h, I.eri, N, 0)[0][0]
    runs = []
    for gamma in (0.0, 0.5):
        dm = sd.DMRG(P, D, seed=3)
        dm.build_boundaries()
        dm.sweep(D, noise=gamma)
        dm.sweep(D, noise=gamma)
        runs.append(np.array(dm.stats.energies))
    n1 = L - 1  # micro-iterations of the first (right) pass
    assert np.allclose(runs[0][:n1], runs[1][:n1], atol=0, rtol=0)
    assert np.abs(runs[0][n1:] - runs[1][n1:]).max() > 0
    assert runs[1].min() >= e_fci - 1e-10
    u = sd.noise_values(3, 1, 2, 1000)
    assert u.min() >= -1.0 and u.max() < 1.0 and abs(u.mean()) < 0.1
