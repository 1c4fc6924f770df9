"""Pins for the oracle's excited states by projection (section "CheMPS2
library", the DMRG object: H_m = H_0 + sum_k eta_k |Psi_k><Psi_k|).

* at the FCI bond dimension the first and second excited states of a
  symmetry sector equal FCI's second and third eigenvalues (S = 0 and 1);
* the projection phi = P_i Psi_k that the solve adds equals the explicit
  projection of the lower state's many-electron vector onto the current
  two-site basis (Fock-space expansion), at a truncated bond dimension.
"""
import numpy as np
import pytest

from oracle import sadmrg as sd
from oracle.explicit import Expansion, Fock, state_vector
from oracle.fci import fci_solve
from synth.integrals import make_integrals


@pytest.mark.parametrize("case", [(6, 6, 0, "C1", 0), (6, 5, 1, "C2", 1), (6, 6, 2, "C1", 0)])
def test_excited_states_equal_fci_roots(case):
    L, N, twoS, group, irrep = case
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    w, _, _ = fci_solve(I.h, I.eri, N, twoS, irrep, I.orb_irrep, nroots=3)
    eta = 2.0 * (w[2] - w[0]) + 1.0
    states = []
    for k in range(3):
        dm = sd.DMRG(P, 400, seed=3 + k)
        dm.build_boundaries()
        for s in states:
            dm.push_lower(s, eta)
        for _ in range(4):
            dm.sweep(400)
        assert abs(dm.emin - w[k]) < 1e-9
        states.append(dm)


def test_projection_equals_the_explicit_projection():
    L, N, twoS, D = 6, 6, 0, 8
    I = make_integrals(L, "C1", 17)
    P = sd.Problem(I.h, I.eri, N, twoS, 0, I.orb_irrep)
    low = sd.DMRG(P, D, seed=4)
    low.build_boundaries()
    low.sweep(D)
    F = Fock(L)
    v_low = state_vector(Expansion(low, F), low).ravel()
    dm = sd.DMRG(P, D, seed=9)
    dm.build_boundaries()
    w = sd.LowerState(low, 1.5)
    for i in range(L - 1):
        El, Er, _, _, secs = dm.enlarged(i)
        ex = Expansion(dm, F)
        B = ex.two_site_basis(i, El, Er, secs, ex.left_states(i), ex.right_states(i + 2))
        phi = sd.project_lower(P, dm, w, i, El, Er, secs)
        for m in secs:
            ref = (B[m] @ v_low).reshape(El.dim[m], Er.dim[m])
            assert np.abs(phi[m] - ref).max() < 1e-12
        if i < L - 2:
            dm.micro(i, D, "right")
