"""The allocation-free sigma entry point (sadmrg_sigma_noalloc) against
sadmrg_sigma on the same prepared steps: two calls in a row, the second on a
smaller input, an in-place call, and the size limit of its static array."""
import numpy as np
import pytest

from oracle import sadmrg as sd
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu


def _ctx(L, N, twoS, group, order, D, step, seed=11):
    from paper_1312_2415_amd import SaDMRG
    I = make_integrals(L, group, seed)
    P = sd.Problem(I.h, I.eri, N, twoS, 0, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    for i in range(step):
        dm.micro(i, D, "right")
    g = SaDMRG(L, order, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, twoS, 0)
    g.mps_import(sd.export_blob(dm))
    g.prepare_step()
    return g


def test_noalloc_sigma_equals_sigma_on_two_calls_in_a_row():
    import torch
    big = _ctx(8, 8, 0, "C1", 1, 40, 3)
    small = _ctx(6, 5, 1, "C1", 1, 10, 1)
    for g, seed in ((big, 1), (small, 2), (big, 3)):
        _, n = g.psi_layout()
        x = torch.from_numpy(np.random.default_rng(seed).normal(size=n)).to("cuda")
        ref = g.sigma(x)
        got = g.sigma_noalloc(x)
        torch.cuda.synchronize()
        err = float((got - ref).abs().max())
        print(f"n={n} max|noalloc - sigma| = {err:.3e}", flush=True)
        assert err <= 1e-13 * float(ref.abs().max())
        xx = x.clone()
        g.sigma_noalloc(xx, xx)  # in place
        assert float((xx - ref).abs().max()) <= 1e-13 * float(ref.abs().max())
    assert small.psi_layout()[1] < big.psi_layout()[1]
    big.close()
    small.close()


def test_noalloc_sigma_rejects_steps_beyond_its_array():
    import torch
    from paper_1312_2415_amd import SaDMRG
    from paper_1312_2415_amd.binding import SadmrgError
    L, D = 14, 800
    I = make_integrals(L, "C1", 7)
    g = SaDMRG(L, 1, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(L, 0, 0)
    g.set_seed(5)
    g.init_mps(D)
    g.advance(D, 6)
    g.prepare_step()
    _, n = g.psi_layout()
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    with pytest.raises(SadmrgError, match="bytes of workspace"):
        g.sigma_noalloc(x)
    y = g.sigma(x)  # the ordinary entry point is unaffected
    assert torch.isfinite(y).all()
    g.close()
