"""Pins for the oracle's reduced density matrices and for the centre move.

* The explicit-expansion RDMs (Fock-space vectors of the MPS, oracle/explicit)
  equal brute-force FCI's at a complete bond dimension: gamma, Gamma^A and the
  multiplet-averaged Gamma^B, for S = 0, 1/2, 1 (paper, calc2DM).
* For a truncated MPS: <S^2> evaluated with the spin operators is S(S+1), and
  equals the value from Gamma^A; tr gamma = N; sum Gamma^A_{ij;ij} = N(N-1);
  Gamma^B obeys the SU(2) relation of a multiplet average; the energy from the
  RDMs equals <Psi|H|Psi>.
* The two-site object moved to the next centre (eqs. StoTT and TTtoS: SVD,
  then recoupling with the next site tensor) represents the same many-electron
  state when nothing is truncated, and loses exactly the discarded weight when
  something is; its Rayleigh quotient with the next step's effective
  Hamiltonian is the previous energy.
"""
import numpy as np
import pytest

from oracle import sadmrg as sd
from oracle.explicit import Expansion, Fock, rdms_of_state, state_vector
from oracle.fci import fci_solve, rdm_b_multiplet, rdms, s2_from_gamma
from synth.integrals import make_integrals


def _dmrg(L, N, twoS, group, irrep, D, seed=11, sweeps=0):
    I = make_integrals(L, group, seed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    for _ in range(sweeps):
        dm.sweep(D)
    return I, P, dm


def _energy_from_rdms(I, g1, GA):
    # E = E_const + sum h_ij gamma_ij + 1/2 sum_ijkl Gamma^A_{ij;kl} (ik|jl)
    return I.e_const + np.einsum("ij,ij->", I.h, g1) + 0.5 * np.einsum("ijkl,ikjl->", GA, I.eri)


@pytest.mark.parametrize("case", [(6, 6, 0, "C1", 0), (5, 5, 1, "C2v", 1), (6, 4, 2, "D2h", 0)])
def test_explicit_rdms_equal_fci_at_complete_bond_dimension(case):
    L, N, twoS, group, irrep = case
    I, P, dm = _dmrg(L, N, twoS, group, irrep, 400, sweeps=2)
    F = Fock(L)
    Psi = state_vector(Expansion(dm, F), dm)
    g1, GA, GB, s2 = rdms_of_state(F, Psi)
    w, v, f = fci_solve(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    fg1, fGA = rdms(f, v[:, 0])
    fGB = rdm_b_multiplet(f, v[:, 0])
    assert abs(dm.emin - w[0]) < 1e-10
    assert np.abs(g1 - fg1).max() < 1e-9
    assert np.abs(GA - fGA).max() < 1e-9
    assert np.abs(GB - fGB).max() < 1e-9
    assert abs(s2 - 0.25 * twoS * (twoS + 2)) < 1e-10
    assert abs(_energy_from_rdms(I, g1, GA) - w[0]) < 1e-10


@pytest.mark.parametrize("case", [(6, 6, 0, "C1", 0, 6), (6, 5, 1, "C2", 1, 5), (7, 6, 2, "C1", 0, 8)])
def test_truncated_mps_rdm_identities(case):
    L, N, twoS, group, irrep, D = case
    I, P, dm = _dmrg(L, N, twoS, group, irrep, D, sweeps=1)
    F = Fock(L)
    Psi = state_vector(Expansion(dm, F), dm)
    g1, GA, GB, s2 = rdms_of_state(F, Psi)
    assert abs(np.trace(g1) - N) < 1e-10
    assert abs(np.einsum("ijij->", GA) - N * (N - 1)) < 1e-9
    # gamma_ik = sum_j Gamma^A_{ij;kj} / (N - 1)
    assert np.abs(np.einsum("ijkj->ik", GA) / (N - 1) - g1).max() < 1e-10
    # the spin-adapted MPS is an exact spin eigenstate, also when truncated
    assert abs(s2 - 0.25 * twoS * (twoS + 2)) < 1e-10
    assert abs(s2_from_gamma(GA, N) - s2) < 1e-10
    # multiplet average: Gamma^B_{ij;kl} = -(Gamma^A_{ij;kl} + 2 Gamma^A_{ij;lk}) / 3
    assert np.abs(GB + (GA + 2.0 * GA.transpose(0, 1, 3, 2)) / 3.0).max() < 1e-10
    # the unsymmetrised Gamma^A is not invariant under i <-> k (it needs its own output)
    assert np.abs(GA - GA.transpose(2, 1, 0, 3)).max() > 1e-3
    H = F.hamiltonian(I.h, I.eri)
    e = float(np.sum(Psi * (H @ Psi)))
    assert abs(_energy_from_rdms(I, g1, GA) - e) < 1e-10


def _move_right(P, dm, i, D):
    psi = dm.center[1]
    U, s, Vt, kept, wd = sd.svd_truncate(psi, D)
    dm.U[i] = U
    dm.dims[i + 1] = kept
    C = {m: s[m][:, None] * Vt[m] for m in kept}
    dm.center = (i + 1, sd.move_center_right(P, C, dm.V[i + 2], i + 1, kept, dm.dims[i + 2]))
    return wd


def _move_left(P, dm, i, D):
    psi = dm.center[1]
    U, s, Vt, kept, wd = sd.svd_truncate(psi, D)
    dm.V[i + 1] = Vt
    dm.dims[i + 1] = kept
    C = {m: U[m] * s[m][None, :] for m in kept}
    dm.center = (i - 1, sd.move_center_left(P, C, dm.U[i - 1], i + 1, kept, dm.dims[i]))
    return wd


@pytest.mark.parametrize("case", [(6, 6, 0, "C1", 0), (6, 5, 1, "C2v", 1), (6, 6, 2, "D2h", 0)])
def test_centre_move_preserves_the_state(case):
    L, N, twoS, group, irrep = case
    I, P, dm = _dmrg(L, N, twoS, group, irrep, 400)
    F = Fock(L)
    H = F.hamiltonian(I.h, I.eri)
    for i in range(L - 2):  # left to right
        dm.micro(i, 400, "right", do_svd=False)
        e = dm.stats.energies[-1]
        v1 = state_vector(Expansion(dm, F), dm)
        n1 = np.sqrt(sum(float(np.sum(x * x)) for x in dm.center[1].values()))
        wd = _move_right(P, dm, i, 400)
        assert wd < 1e-28
        n2 = np.sqrt(sum(float(np.sum(x * x)) for x in dm.center[1].values()))
        assert abs(n1 - n2) < 1e-12 * n1
        v2 = state_vector(Expansion(dm, F), dm)
        assert np.abs(v1 - v2).max() < 1e-12
        assert abs(float(np.sum(v2 * (H @ v2))) - e) < 1e-10
        # the next step's effective Hamiltonian sees the same Rayleigh quotient
        dm.Lblk[i + 1] = sd.renorm_left(dm.enlarged(i)[2], dm.U[i], dm.dims[i + 1])
        El, Er, Xe, Ye, secs = dm.enlarged(i + 1)
        He = sd.Heff(P, Xe, Ye, secs)
        x = dm.center[1]
        hx = He.apply({m: x.get(m, np.zeros((El.dim[m], Er.dim[m]))) for m in secs})
        rq = sum(float(np.sum(x[m] * hx[m])) for m in x) / n2 ** 2
        assert abs(rq - e) < 1e-10
    for i in range(L - 2, 0, -1):  # right to left
        dm.micro(i, 400, "left", do_svd=False)
        v1 = state_vector(Expansion(dm, F), dm)
        wd = _move_left(P, dm, i, 400)
        dm.Rblk[i + 1] = sd.renorm_right(dm.enlarged(i)[3], dm.V[i + 1], dm.dims[i + 1])
        v2 = state_vector(Expansion(dm, F), dm)
        assert wd < 1e-28
        assert np.abs(v1 - v2).max() < 1e-12


def test_truncating_move_loses_the_discarded_weight():
    """|Psi - Psi_trunc|^2 = w_disc for normalised Psi (eq. for w^disc)."""
    I, P, dm = _dmrg(7, 6, 0, "C1", 0, 400)
    F = Fock(7)
    for i in range(3):
        dm.micro(i, 400, "right")
    dm.micro(3, 400, "right", do_svd=False)
    v1 = state_vector(Expansion(dm, F), dm)
    nrm = np.sqrt(sum(float(np.sum(x * x)) for x in dm.center[1].values()))
    dm.center = (3, {m: x / nrm for m, x in dm.center[1].items()})
    wd = _move_right(P, dm, 3, 6)
    assert wd > 1e-6
    ex = Expansion(dm, F)
    Psi_t = state_vector(ex, dm)  # renormalised: compare with the unnormalised projection
    nt = np.sqrt(sum(float(np.sum(x * x)) for x in dm.center[1].values()))
    assert abs(nt ** 2 - (1.0 - wd)) < 1e-12
    assert abs(np.sum((v1 - nt * Psi_t) ** 2) - wd) < 1e-12
