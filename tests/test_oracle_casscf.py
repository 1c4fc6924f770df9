"""Pins for the oracle's CASSCF loop (the DMRG-SCF algorithm with an FCI
active-space solver, section "DMRG-SCF").

* the gradient and the exact Hessian equal finite differences of the energy
  E(kappa) with the RDMs fixed, computed from the plain definition (integrals
  rotated by exp(-kappa), contracted with D and d);
* the full-space RDMs of (closed-shell core) x (active state) reproduce the
  core energy plus the active FCI energy;
* with no active orbitals the loop is restricted Hartree-Fock, checked
  against a plain Roothaan SCF;
* with every orbital active there is nothing to rotate and the energy is FCI;
* the loop converges (gradient below threshold, energy lowered), and an
  initial rotation among the active orbitals (redundant) changes nothing.
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import casscf as cs
from oracle.fci import fci_solve
from synth.integrals import make_integrals


def _case(L=6, seed=21, group="C1"):
    return make_integrals(L, group, seed)


def test_gradient_and_hessian_equal_finite_differences():
    I = _case()
    L = I.L
    C = cs.CASSCF(I.h, I.eri, 0.3, 6, 0, 0, I.orb_irrep, [0, 1, 1, 1, 1, 2])
    R0 = scipy.linalg.expm(-cs.kappa_matrix(L, C.pairs, np.random.default_rng(1).normal(0, 0.1, len(C.pairs))))
    e, h, g, D, d, F = C.step_data(R0)
    assert abs(cs.energy(h, g, D, d, 0.3) - e) < 1e-10
    n = len(C.pairs)

    def E(x):
        h2, g2 = cs.rotate(h, g, scipy.linalg.expm(-cs.kappa_matrix(L, C.pairs, x)))
        return cs.energy(h2, g2, D, d)

    eps = 1e-4
    unit = np.eye(n) * eps
    gfd = np.array([(E(unit[a]) - E(-unit[a])) / (2 * eps) for a in range(n)])
    assert np.abs(gfd - cs.gradient(F, C.pairs)).max() < 1e-7
    H = cs.hessian(h, g, D, d, F, C.pairs)
    Hfd = np.array([[(E(unit[a] + unit[b]) - E(unit[a] - unit[b]) - E(-unit[a] + unit[b]) + E(-unit[a] - unit[b]))
                     / (4 * eps * eps) for b in range(n)] for a in range(n)])
    assert np.abs(H - H.T).max() < 1e-12
    assert np.abs(H - Hfd).max() < 1e-5 * max(1.0, np.abs(H).max())


def _rhf(h, eri, nocc, iters=500):
    """Plain Roothaan SCF in an orthonormal basis (aufbau: lowest nocc
    orbitals of the Fock matrix of the previous density), to convergence."""
    eps, C = np.linalg.eigh(h)
    P = 2.0 * C[:, :nocc] @ C[:, :nocc].T
    for _ in range(iters):
        F = h + np.einsum("rs,pqrs->pq", P, eri) - 0.5 * np.einsum("rs,prsq->pq", P, eri)
        eps, C = np.linalg.eigh(F)
        Pn = 2.0 * C[:, :nocc] @ C[:, :nocc].T
        if np.abs(Pn - P).max() < 1e-13:
            break
        P = Pn
    else:
        raise RuntimeError("SCF did not converge")
    F = h + np.einsum("rs,pqrs->pq", P, eri) - 0.5 * np.einsum("rs,prsq->pq", P, eri)
    return 0.5 * np.einsum("pq,pq->", P, h + F)


def test_no_active_orbitals_is_restricted_hartree_fock():
    # two-electron integrals scaled by 0.1 so that the plain SCF iteration
    # converges (at full strength it oscillates between two densities)
    I = _case(6, 33)
    eri = 0.1 * I.eri
    C = cs.CASSCF(I.h, eri, 0.0, 6, 0, 0, I.orb_irrep, [0, 0, 0, 2, 2, 2])
    hist, R = C.run(grad_tol=1e-10, max_iter=60)
    assert hist[-1][1] < 1e-10
    assert abs(hist[-1][0] - _rhf(I.h, eri, 3)) < 1e-10


def test_all_orbitals_active_is_fci():
    I = _case(5, 7)
    C = cs.CASSCF(I.h, I.eri, 0.0, 4, 2, 0, I.orb_irrep, [1] * 5)
    hist, _ = C.run()
    w, _, _ = fci_solve(I.h, I.eri, 4, 2, 0, I.orb_irrep)
    assert C.pairs == [] and len(hist) == 1
    assert abs(hist[0][0] - w[0]) < 1e-10


@pytest.mark.parametrize("case", [(7, 6, 0, "C1", [0, 1, 1, 1, 1, 2, 2]), (8, 8, 2, "C2v", [0, 0, 1, 1, 1, 1, 1, 2])])
def test_loop_converges_and_ignores_redundant_rotations(case):
    L, N, twoS, group, cls = case
    I = make_integrals(L, group, 5)
    C = cs.CASSCF(I.h, I.eri, 0.0, N, twoS, 0, I.orb_irrep, cls)
    hist, R = C.run(grad_tol=1e-7, max_iter=40)
    assert hist[-1][1] < 1e-7
    assert hist[-1][0] < hist[0][0] - 1e-6
    assert np.abs(R.T @ R - np.eye(L)).max() < 1e-12
    # an initial rotation among active orbitals of one irrep is redundant
    act = [p for p in range(L) if cls[p] == 1 and I.orb_irrep[p] == I.orb_irrep[C.act[0]]]
    K = np.zeros((L, L))
    K[act[0], act[1]], K[act[1], act[0]] = 0.3, -0.3
    hist2, _ = C.run(grad_tol=1e-7, max_iter=40, R0=scipy.linalg.expm(K))
    assert abs(hist2[0][0] - hist[0][0]) < 1e-10
    assert abs(hist2[-1][0] - hist[-1][0]) < 1e-8
