"""Pins for the oracle's SU(2) coefficients.

Clebsch-Gordan coefficients are checked against an independent construction:
diagonalising J^2 in the product basis with explicit ladder operators and
fixing phases by the Condon-Shortley rule.  Coupled-product coefficients are
checked against explicit matrix products in the magnetic basis, and against
the closed form of the singlet coupling.
"""
import math
import itertools

import numpy as np
import pytest

from oracle import su2


def spin_mats(tj):
    ms = list(range(tj, -tj - 1, -2))  # 2m descending
    n = len(ms)
    jz = np.diag([m / 2 for m in ms])
    jp = np.zeros((n, n))
    for a in range(1, n):
        m = ms[a] / 2
        j = tj / 2
        jp[a - 1, a] = math.sqrt(j * (j + 1) - m * (m + 1))
    return jz, jp, ms


def cg_by_diagonalisation(tj1, tj2):
    z1, p1, m1 = spin_mats(tj1)
    z2, p2, m2 = spin_mats(tj2)
    I1, I2 = np.eye(len(m1)), np.eye(len(m2))
    Jz = np.kron(z1, I2) + np.kron(I1, z2)
    Jp = np.kron(p1, I2) + np.kron(I1, p2)
    Jm = Jp.T
    out = {}
    for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
        # highest weight state of spin J: Jz = J, annihilated by J+
        idx = [a * len(m2) + b for a in range(len(m1)) for b in range(len(m2)) if m1[a] + m2[b] == tJ]
        sub = Jp[:, idx]
        _, s, vt = np.linalg.svd(sub)
        v = vt[-1]
        vec = np.zeros(len(m1) * len(m2))
        vec[idx] = v
        # Condon-Shortley: <j1 j1; j2 (J-j1) | J J> > 0
        a0 = 0
        b0 = m2.index(tJ - tj1) if (tJ - tj1) in m2 else None
        if b0 is not None and abs(vec[a0 * len(m2) + b0]) > 1e-12:
            vec *= np.sign(vec[a0 * len(m2) + b0])
        else:
            # first nonzero component with the largest m1 positive
            nz = [i for i in range(len(vec)) if abs(vec[i]) > 1e-12]
            vec *= np.sign(vec[nz[0]])
        tM = tJ
        while tM >= -tJ:
            for a in range(len(m1)):
                for b in range(len(m2)):
                    if m1[a] + m2[b] == tM:
                        out[(m1[a], m2[b], tJ, tM)] = vec[a * len(m2) + b]
            if tM > -tJ:
                J, M = tJ / 2, tM / 2
                vec = Jm @ vec / math.sqrt(J * (J + 1) - M * (M - 1))
            tM -= 2
    return out


@pytest.mark.parametrize("tj1,tj2", [(1, 1), (2, 1), (1, 2), (2, 2), (3, 2), (4, 1), (3, 3), (5, 2)])
def test_cg_matches_ladder_diagonalisation(tj1, tj2):
    ref = cg_by_diagonalisation(tj1, tj2)
    for (tm1, tm2, tJ, tM), v in ref.items():
        assert abs(su2.cg(tj1, tm1, tj2, tm2, tJ, tM) - v) < 1e-12


def test_cg_orthogonality():
    for tj1, tj2 in [(2, 3), (4, 4), (1, 6)]:
        tM = (tj1 + tj2) % 2
        for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
            for tJp in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
                s = sum(su2.cg(tj1, a, tj2, tM - a, tJ, tM) * su2.cg(tj1, a, tj2, tM - a, tJp, tM)
                        for a in range(-tj1, tj1 + 1, 2))
                if tJ >= tM and tJp >= tM:
                    assert abs(s - (tJ == tJp)) < 1e-12


def _tensor(tj_ket, tk, tj_bra, red):
    """Explicit matrix of a rank-k component set with reduced element `red`."""
    mats = {}
    for tq in range(-tk, tk + 1, 2):
        M = np.zeros((tj_bra + 1, tj_ket + 1))
        for i, tm in enumerate(range(-tj_ket, tj_ket + 1, 2)):
            for a, tmp in enumerate(range(-tj_bra, tj_bra + 1, 2)):
                M[a, i] = su2.cg(tj_ket, tm, tk, tq, tj_bra, tmp) * red
        mats[tq] = M
    return mats


def test_same_space_coupling_against_matrix_products():
    rng = np.random.default_rng(0)
    for tj, tjm, tjp, tk1, tk2 in [(1, 0, 1, 1, 1), (1, 2, 1, 1, 1), (2, 1, 2, 1, 1), (2, 3, 4, 1, 1),
                                     (0, 1, 2, 1, 1), (2, 2, 2, 2, 0), (3, 2, 1, 1, 1)]:
        ru, rv = rng.normal(), rng.normal()
        V = _tensor(tj, tk2, tjm, rv)
        U = _tensor(tjm, tk1, tjp, ru)
        for tK in range(abs(tk1 - tk2), tk1 + tk2 + 1, 2):
            if not su2.triangle(tj, tK, tjp):
                continue
            # component Q of [U x V]^K
            for tQ in range(-tK, tK + 1, 2):
                M = sum(su2.cg(tk1, q1, tk2, tQ - q1, tK, tQ) * (U[q1] @ V[tQ - q1])
                        for q1 in range(-tk1, tk1 + 1, 2) if abs(tQ - q1) <= tk2)
                red = su2.same_space_coupling(tj, tjm, tjp, tk1, tk2, tK) * ru * rv
                ref = _tensor(tj, tK, tjp, 1.0)[tQ] * red
                assert np.allclose(M, ref, atol=1e-12)


def test_product_coupling_against_kronecker_products():
    rng = np.random.default_rng(1)
    cases = [(1, 1, 0, 1, 1, 0, 1, 1, 0), (2, 1, 1, 1, 1, 0, 1, 2, 1), (2, 1, 3, 2, 1, 1, 2, 2, 2),
             (3, 0, 3, 1, 1, 0, 2, 1, 3), (1, 1, 2, 1, 1, 2, 0, 0, 0)]
    for (tj1, tj2, tJ, tk1, tk2, tK, tj1p, tj2p, tJp) in cases:
        ra, rb = rng.normal(), rng.normal()
        A = _tensor(tj1, tk1, tj1p, ra)
        B = _tensor(tj2, tk2, tj2p, rb)

        def coupled_states(ta, tb, tJ_):
            S = np.zeros(((ta + 1) * (tb + 1), tJ_ + 1))
            for i, ma in enumerate(range(-ta, ta + 1, 2)):
                for j, mb in enumerate(range(-tb, tb + 1, 2)):
                    for k, M in enumerate(range(-tJ_, tJ_ + 1, 2)):
                        S[i * (tb + 1) + j, k] = su2.cg(ta, ma, tb, mb, tJ_, M)
            return S
        Sk = coupled_states(tj1, tj2, tJ)
        Sb = coupled_states(tj1p, tj2p, tJp)
        for tQ in range(-tK, tK + 1, 2):
            M = sum(su2.cg(tk1, q1, tk2, tQ - q1, tK, tQ) * np.kron(A[q1], B[tQ - q1])
                    for q1 in range(-tk1, tk1 + 1, 2) if abs(tQ - q1) <= tk2)
            got = Sb.T @ M @ Sk
            red = su2.product_coupling(tj1, tj2, tJ, tk1, tk2, tK, tj1p, tj2p, tJp) * ra * rb
            assert np.allclose(got, _tensor(tJ, tK, tJp, 1.0)[tQ] * red, atol=1e-12)


def test_singlet_coupling_closed_form():
    # <(j'j')0||[O^k x P^k]^0||(jj)0> = sqrt((2j'+1)/((2k+1)(2j+1))) for unit reduced elements
    for tj, tjp, tk in itertools.product(range(0, 7), range(0, 7), (0, 1, 2, 3)):
        if su2.triangle(tj, tk, tjp):
            v = su2.product_coupling(tj, tj, 0, tk, tk, 0, tjp, tjp, 0)
            assert abs(v - math.sqrt((tjp + 1) / ((tk + 1) * (tj + 1)))) < 1e-12
