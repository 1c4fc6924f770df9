"""The DMRG energy as a differentiable function of the integrals.

E(h, V) = <psi|H(h, V)|psi> for the MPS that a solver converges to.  Its
derivatives are the spin-summed reduced density matrices the library returns
as the adjoint of the energy (``SaDMRG.rdm``): dE/dh_pq = gamma_pq and, with
the chemist-notation integrals V[i,k,j,l] = (ik|jl) entering the energy as
1/2 sum V[i,k,j,l] Gamma[i,j,k,l], dE/dV[i,k,j,l] = 1/2 Gamma[i,j,k,l].  At
a converged (variational) state the first-order change of the wavefunction
does not change E, so these are the total derivatives -- the quantities a
DMRG-SCF orbital gradient is built from (section "DMRG-SCF").

Only argument marshalling happens here: the solve and the adjoint run inside
the HIP library; torch holds the tensors.
"""
from __future__ import annotations

import numpy as np
import torch


class DMRGEnergy(torch.autograd.Function):
    """``E = DMRGEnergy.apply(h, eri, solver, schedule, e_const, warm)``

    h [L, L] and eri [L, L, L, L] (chemist (ij|kl), eightfold symmetric) are
    float64 tensors on any device; solver is a ``SaDMRG`` with its target set;
    schedule is the ``SaDMRG.solve`` list of (D, e_conv, max_sweeps[, noise]).
    warm: start from the solver's current MPS when it has one (else a new
    random MPS at the first D).  Returns E (0-d float64 tensor, on h's device)
    = e_const + <psi|H|psi> of the final MPS."""

    @staticmethod
    def forward(ctx, h, eri, solver, schedule, e_const=0.0, warm=True):
        blob = None
        if warm:
            try:
                blob = solver.mps_export()
            except Exception:  # no MPS yet
                blob = None
        solver.set_integrals(h.detach().to("cpu", torch.float64).numpy(),
                             eri.detach().to("cpu", torch.float64).numpy(), float(e_const))
        if blob is not None:
            solver.mps_import(blob)
        else:
            solver.init_mps(int(schedule[0][0]))
        solver.solve(schedule)
        g1, g2, e = solver.rdm(two_body=True)
        ctx.save_for_backward(torch.from_numpy(np.ascontiguousarray(g1)).to(h.device),
                              torch.from_numpy(np.ascontiguousarray(g2.transpose(0, 2, 1, 3))).to(h.device))
        return torch.tensor(e, dtype=torch.float64, device=h.device)

    @staticmethod
    def backward(ctx, grad_e):
        g1, g2v = ctx.saved_tensors
        return grad_e * g1, 0.5 * grad_e * g2v, None, None, None, None


def dmrg_energy(h, eri, solver, schedule, e_const=0.0, warm=True):
    """Functional form of ``DMRGEnergy.apply``."""
    return DMRGEnergy.apply(h, eri, solver, schedule, e_const, warm)


def rotate_integrals(h, eri, kappa):
    """The integrals in the orbitals rotated by U = exp(kappa - kappa^T):
    h' = U^T h U and (pq|rs)' = sum_ijkl U_ip U_jq U_kr U_ls (ij|kl)
    (sadmrg_rotation and sadmrg_rotate_integrals in the library; float64
    tensors in, CPU tensors out)."""
    from .binding import rotate_integrals as _rot, rotation
    k = kappa.detach().to("cpu", torch.float64).numpy()
    u = rotation(k - k.T)
    h2, v2 = _rot(u, h.detach().to("cpu", torch.float64).numpy(), eri.detach().to("cpu", torch.float64).numpy())
    return torch.from_numpy(h2), torch.from_numpy(v2)


def orbital_gradient(h, eri, solver, schedule, e_const=0.0):
    """dE/dkappa at kappa = 0 for orbitals rotated by exp(kappa - kappa^T):
    the orbital gradient a DMRG-SCF step (section "DMRG-SCF") is built from.
    The solver re-converges on (h, eri) (warm start), the library returns the
    RDMs (sadmrg_calc2dm) and the orbital gradient 2 (F_pq - F_qp) from the
    generalised Fock matrix (sadmrg_orbital_derivatives, every pair p > q).
    Returns (E, gradient [L, L], antisymmetric)."""
    from .binding import orbital_derivatives
    e = dmrg_energy(h.detach(), eri.detach(), solver, schedule, e_const)
    gchem, _, g1, _, _ = solver.calc2dm(layout=1)
    L = h.shape[0]
    pairs = [(p, q) for p in range(L) for q in range(p)]
    g, _, _ = orbital_derivatives(h.detach().to("cpu", torch.float64).numpy(),
                                  eri.detach().to("cpu", torch.float64).numpy(), g1, gchem, pairs, hessian=False)
    # g_pq = dE/dK_pq for R = exp(-K); kappa - kappa^T = -K
    G = np.zeros((L, L))
    for (p, q), v in zip(pairs, g):
        G[p, q] = -v
        G[q, p] = v
    return e.detach(), torch.from_numpy(G).to(h.device)
