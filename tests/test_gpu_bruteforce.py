"""GPU results against brute force, with no use of the oracle's blocking.

The GPU sigma and the GPU density matrices are compared with the plain
definitions written out in Fock space (oracle/explicit): sigma = P^T H P x
with H built from the unfolded integrals and P the explicit expansion of the
(imported) MPS, and the RDMs as inner products of explicit many-electron
vectors.  Neither side of these comparisons shares the complementary-operator
algebra the GPU path and the oracle's DMRG both implement, so a derivation
error common to the two would show here.  The centre move (section "The
reduced two-site object", eqs. StoTT and TTtoS) is checked through the next
step's initial vector.
"""
import numpy as np
import pytest

from oracle import sadmrg as sd
from oracle.explicit import Expansion, Fock, rdms_of_state, state_vector
from synth.integrals import fourfold_eri, make_integrals

pytestmark = pytest.mark.gpu

ORDER = {"C1": 1, "C2": 2, "C2v": 4, "D2h": 8}
# both pair modes of each block occur along these chains (bare pairs on the
# smaller side), spins 0..2, four point groups, truncated bonds
CASES = [(4, 4, 2, "C1", 0, 16), (5, 5, 1, "C2v", 1, 16), (6, 6, 0, "C1", 0, 6), (6, 5, 3, "C2", 1, 8),
         (6, 6, 4, "D2h", 0, 10), (6, 7, 1, "C2v", 3, 7)]


def _setup(L, N, twoS, group, irrep, D, seed=11, four=False):
    I = make_integrals(L, group, seed)
    if four:  # only (pq|rs) = (rs|pq) = (qp|sr): probes each formula's integral orientation
        I.eri = fourfold_eri(I, seed + 100)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    return I, P, dm


def _gpu(L, group, I, N, twoS, irrep):
    from paper_1312_2415_amd import SaDMRG
    g = SaDMRG(L, ORDER[group], I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, twoS, irrep)
    return g


@pytest.mark.parametrize("four", [False, True])
@pytest.mark.parametrize("case", CASES)
def test_gpu_sigma_equals_projected_hamiltonian(case, four):
    I, P, dm = _setup(*case, four=four)
    L, N, twoS, group, irrep, D = case
    F = Fock(L)
    H = F.hamiltonian(I.h, I.eri)
    g = _gpu(L, group, I, N, twoS, irrep)
    for i in range(L - 1):
        print(f"case {case} step {i}", flush=True)
        g.mps_import(sd.export_blob(dm))
        g.prepare_step()
        desc, n = g.psi_layout()
        ex = Expansion(dm, F)
        El, Er, _, _, secs = dm.enlarged(i)
        assert [tuple(d[:3]) for d in desc] == list(secs)
        B = np.concatenate([v for v in ex.two_site_basis(i, El, Er, secs, ex.left_states(i),
                                                         ex.right_states(i + 2)).values()], axis=0)
        x = np.random.default_rng(200 + i).normal(size=n)
        ref = B @ (H @ (B.T @ x).reshape(F.dim, P.twoS + 1)).ravel()
        got = g.sigma(x)
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
        dref = np.array([b @ (H @ b.reshape(F.dim, P.twoS + 1)).ravel() for b in B])
        assert np.abs(g.heff_diagonal() - dref).max() <= 1e-10 * max(1.0, np.abs(dref).max())
        if i < L - 2:
            dm.micro(i, D, "right")
    g.close()


@pytest.mark.parametrize("case", [(6, 6, 0, "C1", 0, 6, 1), (6, 5, 1, "C2", 1, 5, 1), (7, 6, 2, "C1", 0, 8, 1),
                                  (8, 8, 0, "C1", 0, 12, 0), (8, 7, 3, "C2v", 2, 10, 1)])
def test_gpu_rdms_equal_explicit_rdms_of_a_truncated_mps(case):
    """RDMs of the oracle's MPS at a truncated bond dimension (after a sweep,
    or the random initial state), imported on the GPU, against the explicit
    expansion of the same MPS."""
    L, N, twoS, group, irrep, D, nsw = case
    I, P, dm = _setup(L, N, twoS, group, irrep, D)
    for _ in range(nsw):
        dm.sweep(D)
    F = Fock(L)
    Psi = state_vector(Expansion(dm, F), dm)
    g1, GA, GB, s2_ref = rdms_of_state(F, Psi)
    # <Psi|H|Psi> through the explicit RDMs (the identity is pinned on the CPU
    # against the explicit Hamiltonian, which is slow to build at L = 8)
    e_ref = I.e_const + np.einsum("ij,ij->", I.h, g1) + 0.5 * np.einsum("ijkl,ikjl->", GA, I.eri)
    print(f"case {case}: explicit RDMs done", flush=True)
    g = _gpu(L, group, I, N, twoS, irrep)
    g.mps_import(sd.export_blob(dm))
    ga, gb, r1, s2, e = g.calc2dm()
    g.close()
    assert abs(e - e_ref) < 1e-10
    assert np.abs(r1 - g1).max() < 1e-10
    assert np.abs(ga - GA).max() < 1e-10
    assert np.abs(gb - GB).max() < 1e-10
    assert abs(s2 - s2_ref) < 1e-10


@pytest.mark.parametrize("case", [(6, 6, 0, "C1", 0), (6, 5, 1, "C2v", 1), (7, 8, 2, "D2h", 0)])
def test_gpu_centre_move_keeps_the_state(case):
    """Advancing one step without truncation moves the optimised two-site
    object to the next centre: the next step's initial vector has the
    Rayleigh quotient of the energy just found, and equals the oracle's moved
    object (up to the eigenvector's sign) element by element."""
    L, N, twoS, group, irrep = case
    D = 1000
    I, P, dm = _setup(L, N, twoS, group, irrep, D)
    g = _gpu(L, group, I, N, twoS, irrep)
    g.set_davidson(1e-12, 32, 400)
    dm.dav_tol = 1e-12
    dm.dav_max_iter = 400
    g.mps_import(sd.export_blob(dm))
    for i in range(L - 2):
        print(f"case {case} step {i}", flush=True)
        g.advance(D, 1)
        e_gpu = g.trace()[-1]
        dm.micro(i, D, "right")
        g.prepare_step()
        desc, n = g.psi_layout()
        x = g.guess()
        secs = [tuple(int(v) for v in d[:3]) for d in desc]
        El, Er, _, _, osecs = dm.enlarged(i + 1)
        assert secs == list(osecs)
        ref = np.concatenate([dm.center[1].get(m, np.zeros((El.dim[m], Er.dim[m]))).ravel() for m in secs])
        assert abs(np.linalg.norm(x) - np.linalg.norm(ref)) < 1e-9 * np.linalg.norm(ref)
        sgn = 1.0 if x @ ref >= 0 else -1.0
        assert np.abs(sgn * x - ref).max() < 1e-7 * np.abs(ref).max()
        rq = float(x @ g.sigma(x)) / float(x @ x)
        assert abs(rq - e_gpu) < 1e-10
    g.close()
