"""Pins for the brute-force FCI tool: closed forms and exact identities."""
import math

import numpy as np
import pytest

from oracle.fci import DetSpace, fci_solve, rdms, s2_from_gamma
from synth.integrals import make_integrals


def test_config1_dimension():
    # L=8, N=8, M_S=0: C(8,4)^2 = 4900 determinants (the workload's stated FCI size)
    assert len(DetSpace(8, 8, 0).dets) == 4900


def test_one_body_only_closed_form():
    rng = np.random.default_rng(3)
    L = 6
    A = rng.normal(size=(L, L))
    h = 0.5 * (A + A.T)
    eri = np.zeros((L, L, L, L))
    eps = np.linalg.eigvalsh(h)
    # closed shell singlet, N=4: doubly occupy the two lowest orbitals
    w, _, _ = fci_solve(h, eri, 4, 0)
    assert abs(w[0] - 2 * (eps[0] + eps[1])) < 1e-10
    # doublet N=3: two doubly... lowest is eps0 doubly + eps1 singly
    w, _, _ = fci_solve(h, eri, 3, 1)
    assert abs(w[0] - (2 * eps[0] + eps[1])) < 1e-10
    # triplet N=2: eps0 + eps1 (one in each)
    w, _, _ = fci_solve(h, eri, 2, 2)
    assert abs(w[0] - (eps[0] + eps[1])) < 1e-10


@pytest.mark.parametrize("U,t", [(4.0, 1.0), (1.0, 0.3), (8.0, 2.0)])
def test_hubbard_dimer(U, t):
    h = np.array([[0.0, -t], [-t, 0.0]])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = U
    w, _, _ = fci_solve(h, eri, 2, 0)
    assert abs(w[0] - (U - math.sqrt(U * U + 16 * t * t)) / 2) < 1e-12
    # the triplet of the dimer has energy 0 (no double occupancy, no hopping gain)
    w, _, _ = fci_solve(h, eri, 2, 2)
    assert abs(w[0]) < 1e-12


@pytest.mark.parametrize("N,twoS,group,irrep", [(6, 0, "C1", 0), (5, 1, "C2v", 1), (6, 2, "D2h", 0), (4, 4, "C1", 0)])
def test_rdm_identities_and_spin(N, twoS, group, irrep):
    I = make_integrals(6, group, 77)
    w, v, f = fci_solve(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    g1, G = rdms(f, v[:, 0])
    assert abs(np.trace(g1) - N) < 1e-10
    # N(N-1) = sum_ij Gamma^A_{ij;ij}
    assert abs(np.einsum("ijij->", G) - N * (N - 1)) < 1e-9
    # 1-RDM = sum_j Gamma^A_{ij;kj} / (N-1)
    assert np.allclose(np.einsum("ijkj->ik", G) / (N - 1), g1, atol=1e-10)
    # E = sum h g1 + 1/2 sum Gamma^A_{ij;kl} (ik|jl)
    E = np.einsum("pq,pq->", I.h, g1) + 0.5 * np.einsum("ijkl,ikjl->", G, I.eri)
    assert abs(E - w[0]) < 1e-9
    # spin is exact: <S^2> = S(S+1) from Gamma^A
    S = twoS / 2
    assert abs(s2_from_gamma(G, N) - S * (S + 1)) < 1e-9
    # Gamma^A symmetries
    assert np.allclose(G, G.transpose(1, 0, 3, 2), atol=1e-12)
    assert np.allclose(G, G.transpose(2, 3, 0, 1), atol=1e-12)


def test_variational_penalty_isolates_spin():
    I = make_integrals(5, "C1", 5)
    w0, _, _ = fci_solve(I.h, I.eri, 4, 0)
    w2, _, _ = fci_solve(I.h, I.eri, 4, 2)
    w4, _, _ = fci_solve(I.h, I.eri, 4, 4)
    # each is an eigenvalue of H in the M_S=0 space
    wall, _, _ = fci_solve(I.h, I.eri, 4, 0, nroots=1, mu=0.0)
    # the M_S=0 space holds every spin: its ground state is the lowest of the three
    assert abs(wall[0] - min(w0[0], w2[0], w4[0])) < 1e-9
    assert len({round(w0[0], 8), round(w2[0], 8), round(w4[0], 8)}) == 3
