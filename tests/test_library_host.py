"""Host-side checks of the C-ABI library (no GPU compute)."""
import itertools
import os
import re

import pytest

from oracle import su2
from paper_1312_2415_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _lib():
    if not os.path.exists(binding.library_path()):
        pytest.skip("libsadmrg.so not built")
    return binding.load_library()


def test_exports_every_declared_symbol():
    lib = _lib()
    hdr = open(os.path.join(ROOT, "include", "sadmrg.h")).read()
    names = sorted(set(re.findall(r"\b(sadmrg_[a-z0-9_]+)\s*\(", hdr)))
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n


def test_ninej_product_coupling_matches_cg_definition():
    _lib()
    n = 0
    for tj1, tj2, tk1, tk2, tK in itertools.product(range(0, 5), range(0, 3), range(0, 3), range(0, 3), range(0, 3)):
        for tJ in range(abs(tj1 - tj2), tj1 + tj2 + 1, 2):
            for tj1p in range(abs(tj1 - tk1), tj1 + tk1 + 1, 2):
                for tj2p in range(abs(tj2 - tk2), tj2 + tk2 + 1, 2):
                    for tJp in range(abs(tJ - tK), tJ + tK + 1, 2):
                        a = (tj1, tj2, tJ, tk1, tk2, tK, tj1p, tj2p, tJp)
                        assert abs(binding.debug_coupling(0, a) - su2.product_coupling(*a)) < 1e-12
                        n += 1
    assert n > 1000


def test_sixj_same_space_coupling_matches_cg_definition():
    _lib()
    for tj, tjm, tjp, tk1, tk2, tK in itertools.product(range(0, 6), range(0, 6), range(0, 6), range(0, 3),
                                                         range(0, 3), range(0, 4)):
        a = (tj, tjm, tjp, tk1, tk2, tK)
        assert abs(binding.debug_coupling(1, a) - su2.same_space_coupling(*a)) < 1e-12


def test_sixj_special_values():
    _lib()
    # {a b c; 0 c b} = (-1)^(a+b+c) / sqrt((2b+1)(2c+1))
    for ta, tb, tc in itertools.product(range(0, 7), repeat=3):
        if su2.triangle(ta, tb, tc):
            ref = (-1) ** ((ta + tb + tc) // 2) / ((tb + 1) * (tc + 1)) ** 0.5
            assert abs(binding.debug_coupling(2, (ta, tb, tc, 0, tc, tb)) - ref) < 1e-12
    # orthogonality: sum_x (2x+1)(2j+1) {a b x; c d j}{a b x; c d j'} = delta_jj'
    a, b, c, d = 2, 3, 3, 2
    for tj in range(0, 7):
        for tjp in range(0, 7):
            s = sum((tx + 1) * (tj + 1) * binding.debug_coupling(2, (a, b, tx, c, d, tj))
                    * binding.debug_coupling(2, (a, b, tx, c, d, tjp)) for tx in range(0, 8))
            if su2.triangle(a, d, tj) and su2.triangle(c, b, tj) and su2.triangle(a, d, tjp) and su2.triangle(c, b, tjp):
                assert abs(s - (tj == tjp)) < 1e-12


def test_create_rejects_bad_arguments():
    import ctypes
    lib = _lib()
    h = ctypes.c_void_p()
    irr = (ctypes.c_int * 4)(0, 1, 2, 3)
    assert lib.sadmrg_create(ctypes.byref(h), 1, 1, irr, 0) == -1       # L < 2
    assert lib.sadmrg_create(ctypes.byref(h), 4, 3, irr, 0) == -1       # bad group order
    assert lib.sadmrg_create(ctypes.byref(h), 4, 2, irr, 0) == -1       # irrep out of range


def test_discarded_weight_fit():
    """E(D) = E0 + C1 w(D) (section "Extrapolation"): a line is recovered
    exactly, noisy pairs give the least-squares line, an exact (w = 0)
    energy is returned as it is, a single pair carries no slope."""
    import numpy as np
    pts = [(w, -1.5 + 3.0 * w) for w in (1e-3, 4e-4, 1e-4)]
    e0, c1 = binding.fit_discarded_weight(pts)
    assert abs(e0 + 1.5) <= 1e-12 and abs(c1 - 3.0) <= 1e-9
    rng = np.random.default_rng(1)
    w = np.array([2e-3, 1e-3, 5e-4, 2e-4])
    e = -2.0 + 5.0 * w + rng.normal(scale=1e-5, size=w.size)
    e0, c1 = binding.fit_discarded_weight(list(zip(w, e)))
    c1_ref, e0_ref = np.polyfit(w, e, 1)
    assert abs(e0 - e0_ref) <= 1e-10 and abs(c1 - c1_ref) <= 1e-6
    assert binding.fit_discarded_weight([(1e-3, -1.0), (0.0, -1.2), (0.0, -1.1)]) == (-1.2, 0.0)
    assert binding.fit_discarded_weight([(1e-3, -1.0)]) == (-1.0, 0.0)
    with pytest.raises(ValueError):
        binding.fit_discarded_weight([])


def test_bench_runs_on_one_gpu_only():
    """bench.py measures one GPU: a request for more exits with a message before any GPU work."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
    assert r.stdout.strip() == ""  # no JSON line
