"""Independent problems swept in lockstep (sadmrg_batch_sweep).

Several contexts with different sizes, targets, point groups and bond
dimensions share each Davidson iteration's sigma launches.  Every context's
energies must equal the oracle's sweep of the same problem from the same
initial MPS (1e-8 E_h, as for single sweeps); a batch of one runs exactly
the single-context path; mixed precision stays within 1e-6 E_h of the FP64
oracle; FCI-sized instances reach the exact energy; and malformed batches
are rejected before any work.
"""
import numpy as np
import pytest

from oracle import sadmrg as sd
from oracle.fci import fci_solve
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu

ORDER = {"C1": 1, "C2": 2, "C2v": 4, "D2h": 8}

# (L, N, 2S, group, irrep, D, integral seed): uneven sizes and sectors
CASES = [
    (6, 6, 0, "D2h", 0, 12, 21),
    (8, 6, 2, "C2v", 1, 24, 22),
    (10, 10, 0, "D2h", 0, 30, 23),
    (7, 8, 0, "C1", 0, 16, 24),
    (9, 8, 4, "C2", 1, 20, 25),
]


def _pair(case, seed=3):
    """(oracle DMRG, GPU solver) for one problem, both at the same initial MPS."""
    from paper_1312_2415_amd import SaDMRG
    L, N, twoS, group, irrep, D, iseed = case
    I = make_integrals(L, group, iseed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=seed)
    dm.build_boundaries()
    g = SaDMRG(L, ORDER[group], I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, twoS, irrep)
    g.set_davidson(1e-9, 32, 200)
    g.mps_import(sd.export_blob(dm))
    return dm, g


def test_batched_sweeps_match_oracle_per_instance():
    from paper_1312_2415_amd.binding import batch_sweep
    pairs = [_pair(c) for c in CASES]
    Ds = [c[5] for c in CASES]
    nsw = 2
    for s in range(nsw):
        print(f"batch sweep {s} of {len(CASES)} instances", flush=True)
        em, st, rc = batch_sweep([g for _, g in pairs], Ds)
        assert rc == 0
        assert st["n_sigma"] > 0 and st["flops_sigma"] > 0 and st["t_sigma"] > 0
        for (dm, g), D, e in zip(pairs, Ds, em):
            dm.sweep(D)
            assert abs(e - min(dm.stats.energies[-2 * (dm.P.L - 1):])) <= 1e-8
    for case, (dm, g) in zip(CASES, pairs):
        got, ref = g.trace(), np.array(dm.stats.energies)
        assert len(got) == len(ref), case
        assert np.abs(got - ref).max() <= 1e-8, case
        assert abs(g.energy()[0] - dm.emin) <= 1e-8, case
        g.close()


def test_batch_equals_separate_sweeps_and_batch_of_one_is_the_single_path():
    from paper_1312_2415_amd.binding import batch_sweep
    cases = CASES[:3]
    batched = [_pair(c)[1] for c in cases]
    alone = [_pair(c)[1] for c in cases]
    Ds = [c[5] for c in cases]
    print("batched vs separate", flush=True)
    em, _, _ = batch_sweep(batched, Ds)
    for g, D, e in zip(alone, Ds, em):
        e1, _ = g.sweep(D)
        assert abs(e1 - e) <= 1e-9
    for a, b in zip(batched, alone):
        assert np.abs(a.trace() - b.trace()).max() <= 1e-9
    # a batch of one takes the single-context path: identical bits
    one = _pair(cases[1])[1]
    ref = _pair(cases[1])[1]
    print("batch of one", flush=True)
    e_one, st, _ = batch_sweep([one], [Ds[1]])
    e_ref, _ = ref.sweep(Ds[1])
    assert e_one[0] == e_ref
    assert np.array_equal(one.trace(), ref.trace())
    assert st["n_sigma"] == 0
    for g in batched + alone + [one, ref]:
        g.close()


def test_batched_fci_instances_reach_the_exact_energy():
    from paper_1312_2415_amd import SaDMRG
    from paper_1312_2415_amd.binding import batch_sweep
    specs = [(6, 6, 0, "D2h", 0, 31), (7, 6, 2, "C1", 0, 32), (8, 8, 0, "C2v", 0, 33)]
    gs, efci = [], []
    for L, N, twoS, group, irrep, iseed in specs:
        I = make_integrals(L, group, iseed)
        efci.append(fci_solve(I.h, I.eri, N, twoS, irrep=irrep, orb_irrep=I.orb_irrep)[0][0])
        g = SaDMRG(L, ORDER[group], I.orb_irrep, device=0)
        g.set_integrals(I.h, I.eri)
        g.set_target(N, twoS, irrep)
        g.set_seed(5)
        g.init_mps(200)
        gs.append(g)
    for s in range(3):
        print(f"fci batch sweep {s}", flush=True)
        em, _, _ = batch_sweep(gs, 200)
    for g, e, ef in zip(gs, em, efci):
        assert abs(e - ef) <= 1e-9
        g.close()


def test_mixed_precision_batch_matches_fp64_oracle():
    from paper_1312_2415_amd.binding import batch_sweep
    cases = CASES[1:4]
    pairs = [_pair(c) for c in cases]
    for _, g in pairs:
        g.set_precision(1)
    Ds = [c[5] for c in cases]
    for s in range(2):
        print(f"mixed batch sweep {s}", flush=True)
        em, st, rc = batch_sweep([g for _, g in pairs], Ds)
        assert st["n_sigma32"] > 0 and st["n_sigma"] > 0  # FP32 Davidson, FP64 quotients
        for (dm, _), D in zip(pairs, Ds):
            dm.sweep(D)
    for case, (dm, g) in zip(cases, pairs):
        L = case[0]
        got, ref = g.trace(), np.array(dm.stats.energies)
        assert len(got) == len(ref), case
        # the final pass (the first sweep's truncations may follow the FP32
        # rounding of unconverged states), and the lowest energy
        assert np.abs(got[-(L - 1):] - ref[-(L - 1):]).max() <= 1e-6, case
        assert abs(g.energy()[0] - dm.emin) <= 1e-6, case
        g.close()


def test_mixed_batch_with_refinement_steps():
    """Two FP64 refinement steps in a batch (their sigma shared like the
    others): energies on the oracle's; contexts with different refinement
    are not batched together."""
    from paper_1312_2415_amd.binding import SadmrgError, batch_sweep
    cases = CASES[1:3]
    pairs = [_pair(c) for c in cases]
    for _, g in pairs:
        g.set_precision(1)
        g.set_refinement(2)
    Ds = [c[5] for c in cases]
    for s in range(2):
        print(f"refined mixed batch sweep {s}", flush=True)
        batch_sweep([g for _, g in pairs], Ds)
        for (dm, _), D in zip(pairs, Ds):
            dm.sweep(D)
    for case, (dm, g) in zip(cases, pairs):
        L = case[0]
        got, ref = g.trace(), np.array(dm.stats.energies)
        assert len(got) == len(ref), case
        assert np.abs(got[-(L - 1):] - ref[-(L - 1):]).max() <= 1e-6, case
    pairs[1][1].set_refinement(3)
    with pytest.raises(SadmrgError):
        batch_sweep([g for _, g in pairs], Ds)
    for _, g in pairs:
        g.close()


def test_malformed_batches_are_rejected():
    from paper_1312_2415_amd.binding import SadmrgError, batch_sweep
    _, a = _pair(CASES[0])
    _, b = _pair(CASES[1])
    with pytest.raises(SadmrgError):
        batch_sweep([a, a], [12, 12])
    b.set_precision(1)
    with pytest.raises(SadmrgError):
        batch_sweep([a, b], [12, 24])
    b.set_precision(0)
    with pytest.raises(SadmrgError):
        batch_sweep([a, b], [12, 0])
    b.advance(24, 2)  # centre away from the left end
    with pytest.raises(SadmrgError):
        batch_sweep([a, b], [12, 24])
    # nothing ran: a still sweeps from its imported state
    e, _, rc = batch_sweep([a], [12])
    assert rc == 0 and np.isfinite(e[0])
    a.close()
    b.close()
