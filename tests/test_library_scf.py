"""Host arithmetic of the DMRG-SCF loop in the C library, against the
oracle's independent numpy/scipy versions (no GPU work): integral rotation,
the matrix exponential of an antisymmetric generator, and the generalised
Fock matrix, orbital gradient and exact Hessian with the RDMs fixed."""
import os

import numpy as np
import pytest
import scipy.linalg

from oracle import casscf as cs
from paper_1312_2415_amd import binding
from synth.integrals import make_integrals


def _lib():
    if not os.path.exists(binding.library_path()):
        pytest.skip("libsadmrg.so not built")


def test_rotation_and_integral_transformation():
    _lib()
    I = make_integrals(7, "C1", 4)
    rng = np.random.default_rng(3)
    K = rng.normal(0, 0.4, (7, 7))
    K = K - K.T
    R = binding.rotation(K)
    assert np.abs(R - scipy.linalg.expm(K)).max() < 1e-13
    assert np.abs(R.T @ R - np.eye(7)).max() < 1e-14
    h2, g2 = binding.rotate_integrals(R, I.h, I.eri)
    rh, rg = cs.rotate(I.h, I.eri, R)
    assert np.abs(h2 - rh).max() < 1e-12 and np.abs(g2 - rg).max() < 1e-12
    with pytest.raises(binding.SadmrgError):
        binding.rotation(np.ones((3, 3)))  # not antisymmetric


@pytest.mark.parametrize("case", [(6, 6, 0, "C1", [0, 1, 1, 1, 1, 2]), (8, 8, 2, "C2v", [0, 0, 1, 1, 1, 1, 1, 2])])
def test_orbital_derivatives_equal_the_oracle(case):
    _lib()
    L, N, twoS, group, cls = case
    I = make_integrals(L, group, 9)
    C = cs.CASSCF(I.h, I.eri, 0.0, N, twoS, 0, I.orb_irrep, cls)
    rng = np.random.default_rng(5)
    R0 = scipy.linalg.expm(-cs.kappa_matrix(L, C.pairs, rng.normal(0, 0.1, len(C.pairs))))
    e, h, g, D, d, F = C.step_data(R0)
    grad, H, Fl = binding.orbital_derivatives(h, g, D, d, C.pairs)
    assert np.abs(Fl - F).max() < 1e-11
    assert np.abs(grad - cs.gradient(F, C.pairs)).max() < 1e-11
    assert np.abs(H - cs.hessian(h, g, D, d, F, C.pairs)).max() < 1e-10
    with pytest.raises(binding.SadmrgError):
        binding.orbital_derivatives(h, g, D, d, [(L, 0)])
