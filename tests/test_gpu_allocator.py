"""Caller-supplied device allocator (sadmrg_set_allocator): torch's caching
allocator as the context's memory source gives the same sweeps bit for bit,
torch sees the blocks while the context lives and gets them all back when it
is destroyed; misuse and allocation failure are reported."""
import numpy as np
import pytest

from oracle import sadmrg as sd
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu


def _problem():
    I = make_integrals(8, "C1", 1001)
    P = sd.Problem(I.h, I.eri, 8, 0, 0, I.orb_irrep)
    dm = sd.DMRG(P, 24, seed=3)
    dm.build_boundaries()
    return I, sd.export_blob(dm)


def _ctx(I):
    from paper_1312_2415_amd import SaDMRG
    g = SaDMRG(8, 1, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(8, 0, 0)
    g.set_davidson(1e-9, 32, 200)
    return g


def test_torch_caching_allocator_hooks():
    import torch
    I, blob = _problem()
    ref = _ctx(I)
    ref.mps_import(blob)
    ref.sweep(24)
    t_ref = ref.trace()
    ref.close()
    torch.cuda.synchronize()
    base = torch.cuda.memory_allocated()
    calls = {"alloc": 0, "free": 0}
    g = _ctx(I)

    def alloc(n, dev):
        calls["alloc"] += 1
        return torch.cuda.caching_allocator_alloc(n, device=dev)

    def free(p, n, dev):
        calls["free"] += 1
        torch.cuda.caching_allocator_delete(p)

    g.set_allocator(alloc, free)
    g.mps_import(blob)
    g.sweep(24)
    assert calls["alloc"] > 0
    assert torch.cuda.memory_allocated() > base
    assert np.array_equal(g.trace(), t_ref)
    g1, g2, e = g.rdm()
    assert np.isfinite(g2).all()
    g.close()
    torch.cuda.synchronize()
    assert calls["free"] == calls["alloc"]
    assert torch.cuda.memory_allocated() == base


def test_allocator_misuse_and_failure():
    from paper_1312_2415_amd.binding import SadmrgError
    I, blob = _problem()
    g = _ctx(I)
    g.mps_import(blob)
    with pytest.raises(SadmrgError, match="already holds device memory"):
        g.set_allocator(lambda n, d: 0, lambda p, n, d: None)
    g.close()
    g = _ctx(I)
    g.set_allocator(lambda n, d: 0, lambda p, n, d: None)  # every allocation fails
    with pytest.raises(SadmrgError) as ex:
        g.mps_import(blob)
    assert ex.value.code == -4
    g.close()
