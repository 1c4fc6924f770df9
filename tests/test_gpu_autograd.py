"""The DMRG energy as a torch.autograd function of the integrals.

At a bond dimension where DMRG is exact, E(h, V) is the FCI energy, so its
gradient is pinned by central finite differences of the oracle's FCI energy
along random symmetric directions (independent of the GPU path), and the
value by the FCI energy itself.
"""
import numpy as np
import pytest

from oracle.fci import fci_solve
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu


def _direction(L, rng):
    dh = rng.normal(scale=0.05, size=(L, L))
    dh = dh + dh.T
    dv = np.zeros((L,) * 4)
    for _ in range(L):
        b = rng.normal(scale=0.05, size=(L, L))
        b = b + b.T
        dv += np.einsum("ij,kl->ijkl", b, b)
    return dh, dv


def test_energy_gradient_matches_fci_finite_differences():
    import torch
    from paper_1312_2415_amd import SaDMRG
    from paper_1312_2415_amd.autograd import dmrg_energy
    L, N, twoS = 6, 6, 0
    I = make_integrals(L, "C1", 51)
    g = SaDMRG(L, 1, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, twoS, 0)
    g.set_seed(3)
    sched = [(64, 1e-11, 3)]
    h = torch.tensor(I.h, dtype=torch.float64, requires_grad=True)
    v = torch.tensor(I.eri, dtype=torch.float64, requires_grad=True)
    print("forward", flush=True)
    e = dmrg_energy(h, v, g, sched)
    e_fci = fci_solve(I.h, I.eri, N, twoS)[0][0]
    assert abs(float(e.detach()) - e_fci) <= 1e-9
    e.backward()
    gh, gv = h.grad.numpy(), v.grad.numpy()
    assert np.allclose(gh, gh.T, atol=1e-12)
    rng = np.random.default_rng(7)
    tau = 1e-4
    for k in range(3):
        dh, dv = _direction(L, rng)
        ep = fci_solve(I.h + tau * dh, I.eri + tau * dv, N, twoS)[0][0]
        em = fci_solve(I.h - tau * dh, I.eri - tau * dv, N, twoS)[0][0]
        fd = (ep - em) / (2 * tau)
        an = float(np.sum(gh * dh) + np.sum(gv * dv))
        print(f"direction {k}: fd {fd:.10f} adjoint {an:.10f}", flush=True)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd))
    # warm start from the converged MPS on nearby integrals: same FCI energy
    h2 = torch.tensor(I.h + 1e-3 * dh, dtype=torch.float64)
    v2 = torch.tensor(I.eri + 1e-3 * dv, dtype=torch.float64)
    e2 = dmrg_energy(h2, v2, g, sched)
    e2_fci = fci_solve(I.h + 1e-3 * dh, I.eri + 1e-3 * dv, N, twoS)[0][0]
    assert abs(float(e2) - e2_fci) <= 1e-9
    g.close()


def test_orbital_gradient_matches_finite_differences_of_the_frozen_mps_energy():
    """At a truncated bond dimension the energy depends on orbital rotations.
    The orbital gradient from the energy adjoint through the integral
    rotation equals central differences of <psi|H(U(t))|psi> for the frozen
    MPS along random rotation generators (each evaluation rebuilds the
    operators from the MPS with the rotated integrals)."""
    import torch
    from paper_1312_2415_amd import SaDMRG
    from paper_1312_2415_amd.autograd import orbital_gradient, rotate_integrals
    L, N = 6, 6
    I = make_integrals(L, "C1", 52)
    g = SaDMRG(L, 1, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, 0, 0)
    g.set_seed(5)
    sched = [(8, 1e-11, 6)]
    g.init_mps(8)
    g.solve(sched)
    h = torch.tensor(I.h, dtype=torch.float64)
    v = torch.tensor(I.eri, dtype=torch.float64)
    e, grad = orbital_gradient(h, v, g, sched)
    assert torch.allclose(grad, -grad.T, atol=1e-12)
    assert float(grad.abs().max()) > 1e-4  # truncated: the energy is not rotation invariant
    blob = g.mps_export()
    rng = np.random.default_rng(9)
    tau = 2e-5  # E(t) is not linear in t: the quotient's error is O(tau^2)
    for k in range(3):
        K = torch.tensor(rng.normal(size=(L, L)), dtype=torch.float64)
        es = []
        for t in (tau, -tau):
            h2, v2 = rotate_integrals(h, v, t * K)
            g.set_integrals(h2.numpy(), v2.numpy())
            g.mps_import(blob)
            es.append(g.rdm(two_body=False)[2])
        fd = (es[0] - es[1]) / (2 * tau)
        an = float((grad * K).sum())
        print(f"rotation {k}: fd {fd:.12f} adjoint {an:.12f}", flush=True)
        assert abs(fd - an) <= 2e-7 * max(1.0, abs(fd))
    g.close()
