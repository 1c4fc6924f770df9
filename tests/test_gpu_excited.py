"""Excited states by projection on the GPU (sadmrg_push_excitation; section
"CheMPS2 library", the DMRG object) against the oracle: sigma and the
diagonal of H_m = H_0 + sum_k eta_k |Psi_k><Psi_k| at every step of a sweep,
whole excited-state sweeps micro-iteration by micro-iteration, and FCI
roots at the complete bond dimension."""
import numpy as np
import pytest

from oracle import sadmrg as sd
from oracle.fci import fci_solve
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu

ORDER = {"C1": 1, "C2": 2, "C2v": 4, "D2h": 8}


def _gpu(L, group, I, N, twoS, irrep):
    from paper_1312_2415_amd import SaDMRG
    g = SaDMRG(L, ORDER[group], I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, twoS, irrep)
    g.set_davidson(1e-10, 32, 300)
    return g


@pytest.mark.parametrize("case", [(6, 6, 0, "C1", 0, 8), (8, 7, 1, "C2v", 1, 16), (10, 10, 2, "D2h", 0, 30)])
def test_projected_sigma_matches_oracle_at_every_step(case):
    L, N, twoS, group, irrep, D = case
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    low = sd.DMRG(P, D, seed=4)
    low.build_boundaries()
    low.sweep(D)
    low2 = sd.DMRG(P, D, seed=6)
    low2.build_boundaries()
    low2.sweep(D)
    dm = sd.DMRG(P, D, seed=9)
    dm.build_boundaries()
    etas = (1.5, 0.75)
    ws = [sd.LowerState(low, etas[0]), sd.LowerState(low2, etas[1])]
    g = _gpu(L, group, I, N, twoS, irrep)
    g.mps_import(sd.export_blob(low))
    g.push_excitation(etas[0])
    g.mps_import(sd.export_blob(low2))
    g.push_excitation(etas[1])
    for i in range(L - 1):
        print(f"case {case} step {i}", flush=True)
        g.mps_import(sd.export_blob(dm))
        g.prepare_step()
        desc, n = g.psi_layout()
        El, Er, Xe, Ye, secs = dm.enlarged(i)
        assert [tuple(d[:3]) for d in desc] == list(secs)
        He = sd.Heff(P, Xe, Ye, secs)
        shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
        phis = [(w.eta, sd.flatten(sd.project_lower(P, dm, w, i, El, Er, secs), secs)) for w in ws]
        x = np.random.default_rng(400 + i).normal(size=n)
        ref = sd.flatten(He.apply(sd.unflatten(x, shapes, secs)), secs)
        dref = sd.flatten(He.diagonal(shapes), secs)
        for eta, f in phis:
            ref = ref + eta * (f @ x) * f
            dref = dref + eta * f * f
        assert max(np.abs(f).max() for _, f in phis) > 1e-3  # the projections are not empty
        got = g.sigma(x)
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
        assert np.abs(g.heff_diagonal() - dref).max() <= 1e-10 * max(1.0, np.abs(dref).max())
        if i < L - 2:
            dm.micro(i, D, "right")
    g.close()


@pytest.mark.parametrize("case", [(8, 8, 0, "C1", 0, 24, 2), (8, 6, 2, "D2h", 0, 400, 3)])
def test_excited_sweeps_match_oracle(case):
    """Truncated (D = 24) and complete (D = 400: FCI roots) bond dimensions."""
    L, N, twoS, group, irrep, D, nsw = case
    I = make_integrals(L, group, 23)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    eta = 3.0
    ground = sd.DMRG(P, D, seed=3)
    ground.build_boundaries()
    for _ in range(nsw):
        ground.sweep(D)
    exc = sd.DMRG(P, D, seed=8)
    exc.build_boundaries()
    exc.push_lower(ground, eta)
    start = sd.export_blob(exc)
    for _ in range(nsw):
        exc.sweep(D)
    g = _gpu(L, group, I, N, twoS, irrep)
    g.mps_import(sd.export_blob(ground))
    g.push_excitation(eta)
    g.mps_import(start)
    for s in range(nsw):
        print(f"case {case} sweep {s}", flush=True)
        g.sweep(D)
    got, ref = g.trace(), np.array(exc.stats.energies)
    assert len(got) == len(ref)
    assert np.abs(got - ref).max() <= 1e-8
    if D >= 400:
        w, _, _ = fci_solve(I.h, I.eri, N, twoS, irrep, I.orb_irrep, nroots=2)
        assert abs(ground.emin - w[0]) < 1e-9
        assert abs(g.energy()[0] - w[1]) < 1e-8
    # the density matrices are the excited state's own (H_0)
    g1, g2, e = g.rdm()
    assert abs(np.trace(g1) - N) < 1e-9
    g.clear_excitations()
    g.close()


def test_push_needs_a_left_end_centre():
    from paper_1312_2415_amd.binding import SadmrgError
    I = make_integrals(6, "C1", 3)
    g = _gpu(6, "C1", I, 6, 0, 0)
    g.init_mps(8)
    g.advance(8, 2)
    with pytest.raises(SadmrgError):
        g.push_excitation(1.0)
    with pytest.raises(SadmrgError):
        g.push_excitation(-1.0)
    g.close()
