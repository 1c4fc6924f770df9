"""Davidson iterations replayed from a recorded HIP graph
(sadmrg_set_davidson_graph).

The recorded sequence reads every solve's subspace size and flags from
device memory and does the host-driven loop's arithmetic step for step, so
a sweep with it equals the same sweep driven from the host bit for bit:
single contexts in FP64 and FP32, with subspace restarts, with the
iteration limit reached, with excited-state projectors, and lockstep
batches in FP64 and mixed precision.  The sweeps stay on the oracle's.
"""
import numpy as np
import pytest

from oracle import sadmrg as sd
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu

ORDER = {"C1": 1, "C2": 2, "C2v": 4, "D2h": 8}


def _solver(case, blob, replays, prec=0, max_sub=32, max_iter=200):
    from paper_1312_2415_amd import SaDMRG
    L, N, twoS, group, irrep, D, iseed = case
    I = make_integrals(L, group, iseed)
    g = SaDMRG(L, ORDER[group], I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, twoS, irrep)
    g.set_davidson(1e-9, max_sub, max_iter)
    g.set_davidson_graph(replays)
    if prec:
        g.set_precision(prec, 1e-5)
    g.mps_import(blob)
    return g


def _oracle(case, seed=3):
    L, N, twoS, group, irrep, D, iseed = case
    I = make_integrals(L, group, iseed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=seed)
    dm.build_boundaries()
    return dm


CASE = (10, 6, 2, "D2h", 0, 24, 5)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_recorded_iterations_equal_host_driven_sweeps(prec):
    dm = _oracle(CASE)
    blob = sd.export_blob(dm)
    host = _solver(CASE, blob, 0, prec)
    rec = _solver(CASE, blob, 3, prec)
    for s in range(2):
        print(f"precision {prec} sweep {s}", flush=True)
        e0, _ = host.sweep(CASE[5])
        e1, _ = rec.sweep(CASE[5])
        assert e0 == e1
        dm.sweep(CASE[5])
    assert np.array_equal(host.trace(), rec.trace())
    st = rec.stats_graph()
    assert st["records"] > 0 and st["sigma_calls"] > 0 and st["replays"] >= st["records"]
    assert host.stats_graph()["records"] == 0
    ref = np.array(dm.stats.energies)
    if prec == 0:
        assert np.abs(rec.trace() - ref).max() <= 1e-8
    else:  # reduced precision: the final pass and the lowest energy, as for host-driven sweeps
        L = CASE[0]
        assert np.abs(rec.trace()[-(L - 1):] - ref[-(L - 1):]).max() <= 1e-6
        assert abs(rec.energy()[0] - dm.emin) <= 1e-6
    host.close()
    rec.close()


@pytest.mark.parametrize("max_sub,max_iter", [(4, 200), (32, 3)])
def test_restarts_and_iteration_limit_equal_host_driven(max_sub, max_iter):
    """A subspace of four vectors restarts from the Ritz vector inside the
    recording; three iterations stop at the limit with the previous Ritz
    vector.  Both exactly as the host-driven loop."""
    dm = _oracle(CASE)
    blob = sd.export_blob(dm)
    host = _solver(CASE, blob, 0, max_sub=max_sub, max_iter=max_iter)
    rec = _solver(CASE, blob, 2, max_sub=max_sub, max_iter=max_iter)
    print(f"max_sub {max_sub} max_iter {max_iter}", flush=True)
    host.sweep(CASE[5])
    rec.sweep(CASE[5])
    assert np.array_equal(host.trace(), rec.trace())
    host.close()
    rec.close()


def test_excited_state_projectors_inside_the_recording():
    dm = _oracle(CASE)
    low = _oracle(CASE, seed=4)
    low.sweep(CASE[5])
    gs = []
    for replays in (0, 4):
        g = _solver(CASE, sd.export_blob(low), replays)
        g.push_excitation(1.25)
        g.mps_import(sd.export_blob(dm))
        gs.append(g)
    print("excited-state sweeps", flush=True)
    for g in gs:
        g.sweep(CASE[5])
    assert np.array_equal(gs[0].trace(), gs[1].trace())
    for g in gs:
        g.close()


BATCH = [
    (6, 6, 0, "D2h", 0, 12, 21),
    (8, 6, 2, "C2v", 1, 24, 22),
    (10, 10, 0, "D2h", 0, 30, 23),
    (9, 8, 4, "C2", 1, 20, 25),
]


@pytest.mark.parametrize("prec", [0, 1])
def test_recorded_lockstep_batch_equals_host_driven_batch(prec):
    from paper_1312_2415_amd.binding import SadmrgError, batch_sweep
    blobs = [sd.export_blob(_oracle(c)) for c in BATCH]
    host = [_solver(c, b, 0, prec) for c, b in zip(BATCH, blobs)]
    rec = [_solver(c, b, 3, prec) for c, b in zip(BATCH, blobs)]
    Ds = [c[5] for c in BATCH]
    for s in range(2):
        print(f"batch precision {prec} sweep {s}", flush=True)
        e0, _, _ = batch_sweep(host, Ds)
        e1, _, _ = batch_sweep(rec, Ds)
        assert e0 == e1
    for a, b in zip(host, rec):
        assert np.array_equal(a.trace(), b.trace())
        assert b.stats_graph()["records"] > 0
    rec[1].set_davidson_graph(0)  # contexts that differ in it are not batched together
    with pytest.raises(SadmrgError):
        batch_sweep(rec, Ds)
    for g in host + rec:
        g.close()
