"""SU(2) coupling coefficients for the oracle (plain definitions).

Spins are passed doubled (tj = 2j, tm = 2m) so that everything is integer.

* ``cg`` is the Clebsch-Gordan coefficient <j1 m1; j2 m2 | J M> in the
  Condon-Shortley phase convention, from Racah's closed-form sum.
* ``product_coupling`` and ``same_space_coupling`` give the reduced matrix
  elements of coupled operator products.  They are evaluated directly from
  their definition as sums of products of Clebsch-Gordan coefficients over all
  magnetic quantum numbers -- no 6j or 9j symbols are used here, so the oracle
  is independent of the recoupling formulas the GPU path relies on.

Reduced-matrix-element convention (used throughout the oracle): for a tensor
operator T^k,
    <j' m' | T^k_q | j m> = <j m; k q | j' m'> <j' || T^k || j>,
the same ordering as the paper's reduced MPS tensors (section "Reduced MPS
tensors", eq. tensordecomp: left/ket spin first, then the local/operator spin).
"""
from __future__ import annotations

import functools
import math


def _f(n2: int) -> float:
    """factorial of n2/2 where n2 is even and >= 0"""
    assert n2 % 2 == 0 and n2 >= 0
    return math.factorial(n2 // 2)


def triangle(ta: int, tb: int, tc: int) -> bool:
    return abs(ta - tb) <= tc <= ta + tb and (ta + tb + tc) % 2 == 0


@functools.lru_cache(maxsize=None)
def cg(tj1: int, tm1: int, tj2: int, tm2: int, tJ: int, tM: int) -> float:
    """<j1 m1; j2 m2 | J M> (Racah formula)."""
    if tm1 + tm2 != tM:
        return 0.0
    if not triangle(tj1, tj2, tJ):
        return 0.0
    if abs(tm1) > tj1 or abs(tm2) > tj2 or abs(tM) > tJ:
        return 0.0
    if (tj1 + tm1) % 2 or (tj2 + tm2) % 2 or (tJ + tM) % 2:
        return 0.0
    pre = (tJ + 1) * _f(tJ + tj1 - tj2) * _f(tJ - tj1 + tj2) * _f(tj1 + tj2 - tJ) / _f(tj1 + tj2 + tJ + 2)
    pre *= _f(tJ + tM) * _f(tJ - tM) * _f(tj1 - tm1) * _f(tj1 + tm1) * _f(tj2 - tm2) * _f(tj2 + tm2)
    s = 0.0
    for tk in range(0, tj1 + tj2 + tJ + 2, 2):
        a = tj1 + tj2 - tJ - tk
        b = tj1 - tm1 - tk
        c = tj2 + tm2 - tk
        d = tJ - tj2 + tm1 + tk
        e = tJ - tj1 - tm2 + tk
        if min(a, b, c, d, e) < 0:
            continue
        s += (-1) ** (tk // 2) / (_f(tk) * _f(a) * _f(b) * _f(c) * _f(d) * _f(e))
    return math.sqrt(pre) * s


def _ms(tj: int):
    return range(-tj, tj + 1, 2)


@functools.lru_cache(maxsize=None)
def product_coupling(tj1: int, tj2: int, tJ: int, tk1: int, tk2: int, tK: int,
                     tj1p: int, tj2p: int, tJp: int) -> float:
    """Reduced element of [A^{k1} x B^{k2}]^K between coupled two-subsystem states.

    Ket |(j1 j2) J>, bra |(j1' j2') J'>, A acts on subsystem 1 and B on
    subsystem 2, both with unit reduced elements; fermion signs are not
    included.  Evaluated from the definition:
      sum over all m of CG(bra coupling) * CG(A) * CG(B) * CG(K coupling)
      * CG(ket coupling), divided by the Wigner-Eckart CG of the result.
    """
    if not (triangle(tj1, tj2, tJ) and triangle(tj1p, tj2p, tJp) and triangle(tk1, tk2, tK)
            and triangle(tj1, tk1, tj1p) and triangle(tj2, tk2, tj2p) and triangle(tJ, tK, tJp)):
        return 0.0
    # choose the (M, Q, M') with the largest Wigner-Eckart coefficient
    best = None
    for tM in _ms(tJ):
        for tQ in _ms(tK):
            tMp = tM + tQ
            if abs(tMp) > tJp:
                continue
            w = cg(tJ, tM, tK, tQ, tJp, tMp)
            if best is None or abs(w) > abs(best[0]):
                best = (w, tM, tQ, tMp)
    w, tM, tQ, tMp = best
    if abs(w) < 1e-12:
        return 0.0
    tot = 0.0
    for tm1 in _ms(tj1):
        tm2 = tM - tm1
        if abs(tm2) > tj2:
            continue
        c_ket = cg(tj1, tm1, tj2, tm2, tJ, tM)
        if c_ket == 0.0:
            continue
        for tq1 in _ms(tk1):
            tq2 = tQ - tq1
            if abs(tq2) > tk2:
                continue
            c_op = cg(tk1, tq1, tk2, tq2, tK, tQ)
            if c_op == 0.0:
                continue
            tm1p, tm2p = tm1 + tq1, tm2 + tq2
            if abs(tm1p) > tj1p or abs(tm2p) > tj2p:
                continue
            tot += (cg(tj1p, tm1p, tj2p, tm2p, tJp, tMp) * cg(tj1, tm1, tk1, tq1, tj1p, tm1p)
                    * cg(tj2, tm2, tk2, tq2, tj2p, tm2p) * c_op * c_ket)
    return tot / w


@functools.lru_cache(maxsize=None)
def same_space_coupling(tj: int, tjm: int, tjp: int, tk1: int, tk2: int, tK: int) -> float:
    """Coefficient of <j'||U||j''><j''||V||j> in <j'||[U^{k1} x V^{k2}]^K||j>.

    U and V act on the same space (V first); evaluated from the definition by
    summing Clebsch-Gordan coefficients over all projections.
    """
    if not (triangle(tj, tk2, tjm) and triangle(tjm, tk1, tjp) and triangle(tk1, tk2, tK)
            and triangle(tj, tK, tjp)):
        return 0.0
    best = None
    for tM in _ms(tj):
        for tQ in _ms(tK):
            tMp = tM + tQ
            if abs(tMp) > tjp:
                continue
            w = cg(tj, tM, tK, tQ, tjp, tMp)
            if best is None or abs(w) > abs(best[0]):
                best = (w, tM, tQ, tMp)
    w, tM, tQ, tMp = best
    if abs(w) < 1e-12:
        return 0.0
    tot = 0.0
    for tq1 in _ms(tk1):
        tq2 = tQ - tq1
        if abs(tq2) > tk2:
            continue
        c_op = cg(tk1, tq1, tk2, tq2, tK, tQ)
        if c_op == 0.0:
            continue
        tmm = tM + tq2
        if abs(tmm) > tjm:
            continue
        tot += c_op * cg(tj, tM, tk2, tq2, tjm, tmm) * cg(tjm, tmm, tk1, tq1, tjp, tMp)
    return tot / w
