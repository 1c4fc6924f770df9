"""GPU convergence scheme with noise against the oracle.

The noise (section "Convergence scheme": uniform, bounded by 0.5 gamma times
the largest discarded weight of the previous left- or right-sweep, added just
before each decomposition) draws from the counter generator keyed by (seed,
pass, step); both sides implement it from that definition, so whole noisy
schedules must agree micro-iteration by micro-iteration.
"""
import numpy as np
import pytest

from oracle import sadmrg as sd
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("case", [(8, 8, 0, "C1", 1, 12, 1001), (10, 6, 2, "D2h", 8, 16, 5)])
def test_noisy_schedule_matches_oracle(case):
    from paper_1312_2415_amd import SaDMRG
    L, N, twoS, group, order, D, seed = case
    I = make_integrals(L, group, seed)
    P = sd.Problem(I.h, I.eri, N, twoS, 0, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    schedule = [(D, 1e-12, 2, 0.5), (D + 4, 1e-12, 1, 0.0)]
    dm.solve(schedule)
    g = SaDMRG(L, order, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, twoS, 0)
    g.set_seed(3)
    g.set_davidson(1e-9, 32, 200)
    g.mps_import(blob)
    g.solve(schedule)
    got, ref = g.trace(), np.array(dm.stats.energies)
    assert len(got) == len(ref)
    assert np.abs(got - ref).max() <= 1e-8
    assert abs(g.energy()[0] - dm.emin) <= 1e-8
    g.close()


def test_negative_noise_is_rejected():
    from paper_1312_2415_amd import SaDMRG
    from paper_1312_2415_amd.binding import SadmrgError
    I = make_integrals(4, "C1", 3)
    g = SaDMRG(4, 1, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(4, 0, 0)
    with pytest.raises(SadmrgError):
        g.solve([(8, 1e-8, 1, -0.1)])
    g.close()
