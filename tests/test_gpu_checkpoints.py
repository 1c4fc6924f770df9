"""Renormalised operators recomputed instead of stored
(sadmrg_set_block_checkpoints).

Only the blocks at every k-th bond stay in device memory; the others are
rebuilt from the nearest kept block and the MPS tensors when a step or the
energy adjoint needs them.  Sweeps, the RDMs of the energy adjoint and the
frozen-MPS energy after an integral change equal those with every block
stored (up to the rounding of a different enlargement layout), the oracle's
sweeps still match, and fewer blocks (and bytes) are held at once.
"""
import numpy as np
import pytest

from oracle import sadmrg as sd
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu

ORDER = {"C1": 1, "C2": 2, "C2v": 4, "D2h": 8}
CASE = (12, 12, 0, "D2h", 0, 40, 7)


def _pair(case, interval):
    from paper_1312_2415_amd import SaDMRG
    L, N, twoS, group, irrep, D, iseed = case
    I = make_integrals(L, group, iseed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    g = SaDMRG(L, ORDER[group], I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, twoS, irrep)
    g.set_davidson(1e-9, 32, 200)
    g.set_block_checkpoints(interval)
    g.mps_import(sd.export_blob(dm))
    return dm, g, I


@pytest.mark.parametrize("interval", [2, 4])
def test_checkpointed_sweeps_and_rdms_equal_the_stored_ones(interval):
    L, D = CASE[0], CASE[5]
    dm, full, I = _pair(CASE, 0)
    _, ck, _ = _pair(CASE, interval)
    full.stats_reset()
    ck.stats_reset()
    for s in range(2):
        print(f"interval {interval} sweep {s}", flush=True)
        e0, _ = full.sweep(D)
        e1, _ = ck.sweep(D)
        dm.sweep(D)
        assert abs(e0 - e1) <= 1e-10
    a, b = full.trace(), ck.trace()
    assert np.abs(a - b).max() <= 1e-10
    assert np.abs(b - np.array(dm.stats.energies)).max() <= 1e-8
    sf, sc = full.stats_blocks(), ck.stats_blocks()
    assert sf["rebuilt"] == 0 and sc["rebuilt"] > 0
    assert sc["held"] < sf["held"]
    assert sc["max_bytes"] < sf["max_bytes"]
    print("blocks", sf, sc, flush=True)
    # the energy adjoint walks both ends, rebuilding what it needs
    g1a, g2a, ea = full.rdm()
    g1b, g2b, eb = ck.rdm()
    assert abs(ea - eb) <= 1e-11
    assert np.abs(g1a - g1b).max() <= 1e-10
    assert np.abs(g2a - g2b).max() <= 1e-10
    # a frozen-MPS energy after an integral change rebuilds every block
    blob = full.mps_export()
    h2 = I.h + 1e-3 * np.eye(L)
    es = []
    for g in (full, ck):
        g.set_integrals(h2, I.eri)
        g.mps_import(blob)
        es.append(g.rdm(two_body=False)[2])
    assert abs(es[0] - es[1]) <= 1e-11
    full.close()
    ck.close()


def test_checkpoints_switched_on_between_sweeps():
    L, D = CASE[0], CASE[5]
    _, a, _ = _pair(CASE, 0)
    _, b, _ = _pair(CASE, 0)
    a.sweep(D)
    b.sweep(D)
    b.set_block_checkpoints(3)
    print("switched on", flush=True)
    ea, _ = a.sweep(D)
    eb, _ = b.sweep(D)
    assert abs(ea - eb) <= 1e-10
    assert np.abs(a.trace() - b.trace()).max() <= 1e-10
    from paper_1312_2415_amd.binding import SadmrgError
    with pytest.raises(SadmrgError):
        b.set_block_checkpoints(-1)
    a.close()
    b.close()
