"""GPU precision variant: FP32 sigma (FP32 operators, FP32 accumulation) with
FP64 Davidson algebra and an FP64 Rayleigh-quotient energy per micro-iteration.

Checked against the FP64 oracle: the FP32 sigma stays within FP32 rounding of
the oracle's sigma at every step, and mixed-precision sweep energies match
the oracle's FP64 sweep to 1e-6 E_h (the precision target), including an
FCI-exact case.
"""
import numpy as np
import pytest

from oracle import sadmrg as sd
from oracle.fci import fci_solve
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu

ORDER = {"C1": 1, "C2": 2, "C2v": 4, "D2h": 8}


def _gpu(L, group, I):
    from paper_1312_2415_amd import SaDMRG
    g = SaDMRG(L, ORDER[group], I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    return g


@pytest.mark.parametrize("case", [(6, 6, 2, "D2h", 0, 10), (10, 10, 0, "D2h", 0, 30)])
def test_fp32_sigma_within_fp32_rounding_of_oracle(case):
    L, N, twoS, group, irrep, D = case
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    for i in range(L - 1):
        print(f"case {case} step {i}", flush=True)
        g.mps_import(sd.export_blob(dm))
        g.prepare_step()
        desc, n = g.psi_layout()
        El, Er, Xe, Ye, secs = dm.enlarged(i)
        He = sd.Heff(P, Xe, Ye, secs)
        shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
        x = np.random.default_rng(100 + i).normal(size=n)
        ref = sd.flatten(He.apply(sd.unflatten(x, shapes, secs)), secs)
        g.set_precision(1)
        got32 = g.sigma(x)
        g.set_precision(0)
        got64 = g.sigma(x)
        scale = np.abs(ref).max()
        err32 = np.abs(got32 - ref).max() / scale
        assert err32 <= 2e-5
        if n > 8:  # the FP32 path really ran in FP32
            assert err32 > 1e-12
        assert np.abs(got64 - ref).max() <= 1e-10 * scale
        if i < L - 2:
            dm.micro(i, D, "right")
    st = g.stats()
    assert st["fp32"]["calls"] >= L - 1
    g.close()


@pytest.mark.parametrize("case", [(8, 8, 0, "C1", 0, 64, 3, 1001), (10, 6, 2, "D2h", 0, 24, 2, 5),
                                  (12, 12, 0, "D2h", 0, 40, 2, 7)])
def test_mixed_sweep_energies_match_fp64_oracle(case):
    L, N, twoS, group, irrep, D, nsw, seed = case
    I = make_integrals(L, group, seed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    for _ in range(nsw):
        dm.sweep(D)
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    g.set_davidson(1e-9, 32, 200)
    g.set_precision(1, 1e-5)
    g.mps_import(blob)
    for s in range(nsw):
        print(f"case {case} sweep {s}", flush=True)
        g.sweep(D)
    got, ref = g.trace(), np.array(dm.stats.energies)
    assert len(got) == len(ref)
    assert np.abs(got[-(L - 1):] - ref[-(L - 1):]).max() <= 1e-6  # the final sweep
    assert abs(g.energy()[0] - dm.emin) <= 1e-6
    assert g.stats()["fp32"]["calls"] > 0
    if case[0] == 8:  # D = 64 at L = 8 is complete: FCI-exact
        e_fci = fci_solve(I.h, I.eri, N, twoS, irrep, I.orb_irrep, I.e_const, nroots=1)[0][0]
        assert abs(g.energy()[0] - e_fci) <= 1e-6
    g.close()


def test_fp64_refinement_steps():
    """More FP64 Davidson steps after the FP32 phase: one more FP64 sigma per
    step and micro-iteration, energies still on the FP64 oracle's sweeps."""
    from paper_1312_2415_amd.binding import SadmrgError
    L, N, twoS, group, irrep, D, nsw, seed = 10, 6, 2, "D2h", 0, 24, 2, 5
    I = make_integrals(L, group, seed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    for _ in range(nsw):
        dm.sweep(D)
    ref = np.array(dm.stats.energies)
    calls = {}
    for steps in (1, 3):
        g = _gpu(L, group, I)
        g.set_target(N, twoS, irrep)
        g.set_davidson(1e-9, 32, 200)
        g.set_precision(1, 1e-5)
        g.set_refinement(steps)
        g.mps_import(blob)
        g.stats_reset()
        for s in range(nsw):
            print(f"refinement {steps} sweep {s}", flush=True)
            g.sweep(D)
        got = g.trace()
        assert len(got) == len(ref)
        assert np.abs(got[-(L - 1):] - ref[-(L - 1):]).max() <= 1e-6
        assert abs(g.energy()[0] - dm.emin) <= 1e-6
        calls[steps] = g.stats()["n_sigma"] / len(got)  # FP64 sigma per micro-iteration
        for bad in (0, 9):
            with pytest.raises(SadmrgError):
                g.set_refinement(bad)
        g.close()
    assert abs(calls[1] - 2.0) <= 1e-12
    assert 2.0 < calls[3] <= 4.0


def test_refinement_residual_target():
    """With a residual target, FP64 refinement steps after the first run only
    while the refined vector's FP64 residual is above it: BF16x3 Davidson
    (which stops on its rounding floor) then gets the steps it needs, its
    sweeps land closer to the FP64 oracle's than with a single step, and a
    loose target never costs more FP64 sigma than the fixed step count."""
    from paper_1312_2415_amd.binding import SadmrgError
    L, N, twoS, group, irrep, D, nsw, seed = 10, 6, 2, "D2h", 0, 24, 2, 5
    I = make_integrals(L, group, seed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    for _ in range(nsw):
        dm.sweep(D)
    ref = np.array(dm.stats.energies)
    err, calls = {}, {}
    for steps, tol in ((1, 0.0), (6, 1e-8), (6, 1.0)):
        g = _gpu(L, group, I)
        g.set_target(N, twoS, irrep)
        g.set_davidson(1e-9, 32, 200)
        g.set_precision(2, 1e-5)
        g.set_refinement(steps)
        g.set_refinement_tol(tol)
        g.mps_import(blob)
        g.stats_reset()
        for s in range(nsw):
            print(f"refinement {steps} target {tol} sweep {s}", flush=True)
            g.sweep(D)
        got = g.trace()
        assert len(got) == len(ref)
        err[tol] = float(np.abs(got - ref).max())
        calls[tol] = g.stats()["n_sigma"] / len(got)
        with pytest.raises(SadmrgError):
            g.set_refinement_tol(-1.0)
        g.close()
    print(f"max |dE| per micro-iteration: {err}; FP64 sigma per micro-iteration: {calls}", flush=True)
    assert err[1e-8] <= 1e-7
    assert err[1e-8] <= err[0.0]
    assert abs(calls[1.0] - 2.0) <= 1e-12  # the first step only
    assert calls[1e-8] > 2.0


@pytest.mark.parametrize("mode,tol", [(1, 1e-5), (2, 1e-3)])
def test_reduced_precision_renormalisation(mode, tol):
    """Renormalisation products in FP32 (mode 1) or BF16x3 (mode 2): the
    new blocks carry that rounding into every later step, so the sweep
    energies move away from the FP64 oracle's by an amount of the order of
    the products' rounding and stay within `tol` of them (with FP64 sigma,
    and with FP32 sigma in Davidson as well)."""
    from paper_1312_2415_amd.binding import SadmrgError
    L, N, twoS, group, irrep, D, nsw, seed = 10, 6, 2, "D2h", 0, 24, 2, 5
    I = make_integrals(L, group, seed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    for _ in range(nsw):
        dm.sweep(D)
    ref = np.array(dm.stats.energies)
    for sigma_prec in (0, 1):
        g = _gpu(L, group, I)
        g.set_target(N, twoS, irrep)
        g.set_davidson(1e-9, 32, 200)
        if sigma_prec:
            g.set_precision(sigma_prec, 1e-5)
            g.set_refinement(4)
            g.set_refinement_tol(1e-7)
        g.set_renorm_precision(mode)
        g.mps_import(blob)
        for s in range(nsw):
            print(f"renormalisation mode {mode} sigma {sigma_prec} sweep {s}", flush=True)
            g.sweep(D)
        got = g.trace()
        assert len(got) == len(ref)
        err = np.abs(got[-(L - 1):] - ref[-(L - 1):]).max()
        print(f"max |dE| of the final pass {err:.2e}", flush=True)
        assert err <= tol
        assert abs(g.energy()[0] - dm.emin) <= tol
        if sigma_prec == 0:
            assert np.abs(got - ref).max() > 1e-12  # the reduced products really ran
        with pytest.raises(SadmrgError):
            g.set_renorm_precision(3)
        g.close()


def test_bf16x3_sigma_within_its_rounding_of_oracle():
    """Mode 2: BF16x3 products (hi*hi + hi*lo + lo*hi of the BF16 splits,
    FP32 accumulation).  The sigma stays within a few hundred times the
    products' 2^-16 relative rounding of the FP64 oracle, and is measurably
    less exact than the FP32 products (so the BF16 path really ran)."""
    L, N, twoS, group, irrep, D = 10, 10, 0, "D2h", 0, 30
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    worst32 = worst3 = 0.0
    for i in range(L - 1):
        print(f"bf16x3 step {i}", flush=True)
        g.mps_import(sd.export_blob(dm))
        g.prepare_step()
        desc, n = g.psi_layout()
        El, Er, Xe, Ye, secs = dm.enlarged(i)
        He = sd.Heff(P, Xe, Ye, secs)
        shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
        x = np.random.default_rng(200 + i).normal(size=n)
        ref = sd.flatten(He.apply(sd.unflatten(x, shapes, secs)), secs)
        scale = np.abs(ref).max()
        g.set_precision(2)
        e3 = np.abs(g.sigma(x) - ref).max() / scale
        g.set_precision(1)
        e32 = np.abs(g.sigma(x) - ref).max() / scale
        g.set_precision(0)
        assert e3 <= 5e-3
        worst3, worst32 = max(worst3, e3), max(worst32, e32)
        if i < L - 2:
            dm.micro(i, D, "right")
    assert worst3 > 10 * worst32 > 0.0
    g.close()


def test_bf16x3_mixed_sweeps_match_fp64_oracle():
    L, N, twoS, group, irrep, D, nsw, seed = 10, 6, 2, "D2h", 0, 24, 2, 5
    I = make_integrals(L, group, seed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    for _ in range(nsw):
        dm.sweep(D)
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    g.set_davidson(1e-9, 32, 200)
    g.set_precision(2, 1e-5)
    g.mps_import(blob)
    for s in range(nsw):
        print(f"bf16x3 sweep {s}", flush=True)
        g.sweep(D)
    got, ref = g.trace(), np.array(dm.stats.energies)
    assert len(got) == len(ref)
    assert np.abs(got[-(L - 1):] - ref[-(L - 1):]).max() <= 1e-6
    assert abs(g.energy()[0] - dm.emin) <= 1e-6
    assert g.stats()["fp32"]["calls"] > 0
    g.close()


def test_precision_mode_is_validated():
    I = make_integrals(4, "C1", 3)
    g = _gpu(4, "C1", I)
    from paper_1312_2415_amd.binding import SadmrgError
    with pytest.raises(SadmrgError):
        g.set_precision(3)
    with pytest.raises(SadmrgError):
        g.set_precision(-1)
    with pytest.raises(SadmrgError):
        g.set_precision(1, 0.0)
    g.set_precision(1, 1e-6)
    g.set_precision(0)
    g.close()
