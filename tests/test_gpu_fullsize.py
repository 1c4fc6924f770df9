"""Full-size configurations, checked through properties that hold at any size
(the oracle cannot sweep these problems).  The headline shape (L = 28,
N = 12, singlet Ag, D2h, D_SU(2) = 2500) in the launch configuration the
benchmark times:

* H_eff is symmetric in the plain inner product of the TT basis:
  <x|H y> = <y|H x> for random x, y;
* the effective-Hamiltonian diagonal equals <e_i|H e_i> on sampled unit vectors;
* the FP32 and BF16x3 products stay within their rounding of the FP64 sigma;
* the RDMs reproduce the energy: E = e0 + sum h gamma + 1/2 sum (ik|jl) Gamma,
  trace gamma = N, and gamma is symmetric.

The plain FP64 configuration L = 24, N = 12, singlet Ag, D2h, D_SU(2) = 500,
six sweeps: sweep minima do not rise, a larger bond dimension does not raise
the energy, and the same symmetry, diagonal and RDM identities hold.

Both configurations are also compared with the oracle itself at their
middle step: sigma on a deterministic random MPS against stored oracle
values (tests/golden/make_sigma_golden.py).
"""
import numpy as np
import pytest

from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu


def test_headline_shape_properties():
    from paper_1312_2415_amd import SaDMRG
    L, N, D = 28, 12, 2500
    I = make_integrals(L, "D2h", 1003)
    g = SaDMRG(L, 8, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri, I.e_const)
    g.set_target(N, 0, 0)
    g.set_davidson(1e-7, 32, 100)
    g.init_mps(D)
    print("sweep at D=2500", flush=True)
    e_sweep, _ = g.sweep(D)
    assert np.isfinite(e_sweep)
    blob = g.mps_export()
    g.advance(D, L // 2 - 1)
    g.prepare_step()
    desc, n = g.psi_layout()
    assert n > 100000
    rng = np.random.default_rng(12)
    x, y = rng.normal(size=n), rng.normal(size=n)
    print("sigma symmetry", flush=True)
    hx, hy = g.sigma(x), g.sigma(y)
    a, b = float(x @ hy), float(y @ hx)
    assert abs(a - b) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(hy)
    print("diagonal samples", flush=True)
    d = g.heff_diagonal()
    for i in rng.choice(n, 8, replace=False):
        e = np.zeros(n)
        e[i] = 1.0
        assert abs(g.sigma(e)[i] - d[i]) <= 1e-12 * max(1.0, abs(d[i]))
    print("reduced-precision products", flush=True)
    scale = np.abs(hx).max()
    g.set_precision(1)
    e32 = np.abs(g.sigma(x) - hx).max() / scale
    g.set_precision(2)
    e3 = np.abs(g.sigma(x) - hx).max() / scale
    g.set_precision(0)
    assert 0.0 < e32 <= 2e-5
    assert e32 < e3 <= 5e-3
    print("RDM identities", flush=True)
    g.mps_import(blob)
    g1, g2, e = g.rdm()
    e_id = I.e_const + float(np.einsum("pq,pq", I.h, g1)) + 0.5 * float(np.einsum("ikjl,ijkl", I.eri, g2))
    assert abs(e_id - e) <= 1e-9 * max(1.0, abs(e))
    assert abs(np.trace(g1) - N) <= 1e-9
    assert np.abs(g1 - g1.T).max() <= 1e-12
    g.close()


def _symmetry_and_diagonal(g, n, rng, nsamp=6):
    x, y = rng.normal(size=n), rng.normal(size=n)
    hx, hy = g.sigma(x), g.sigma(y)
    assert abs(float(x @ hy) - float(y @ hx)) <= 1e-12 * np.linalg.norm(x) * np.linalg.norm(hy)
    d = g.heff_diagonal()
    for i in rng.choice(n, nsamp, replace=False):
        e = np.zeros(n)
        e[i] = 1.0
        assert abs(g.sigma(e)[i] - d[i]) <= 1e-12 * max(1.0, abs(d[i]))


def test_l24_d500_sweeps_and_identities():
    from paper_1312_2415_amd import SaDMRG
    L, N = 24, 12
    I = make_integrals(L, "D2h", 1002)
    g = SaDMRG(L, 8, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri, I.e_const)
    g.set_target(N, 0, 0)
    g.set_davidson(1e-8, 32, 200)
    g.init_mps(250)
    e250 = min(g.sweep(250)[0] for _ in range(3))
    es = []
    for s in range(6):
        e, _ = g.sweep(500)
        print(f"L=24 D=500 sweep {s}: {e:.10f}", flush=True)
        es.append(e)
    assert all(np.isfinite(es))
    assert all(b <= a + 1e-8 for a, b in zip(es, es[1:]))  # sweep minima do not rise
    assert es[-1] <= e250 + 1e-8  # more states, no higher energy
    blob = g.mps_export()
    g.advance(500, L // 2 - 1)
    g.prepare_step()
    desc, n = g.psi_layout()
    assert n > 10000
    _symmetry_and_diagonal(g, n, np.random.default_rng(24))
    g.mps_import(blob)
    g1, g2, e = g.rdm()
    e_id = I.e_const + float(np.einsum("pq,pq", I.h, g1)) + 0.5 * float(np.einsum("ikjl,ijkl", I.eri, g2))
    assert abs(e_id - e) <= 1e-9 * max(1.0, abs(e))
    assert abs(np.trace(g1) - N) <= 1e-9
    assert np.abs(g1 - g1.T).max() <= 1e-12
    assert e >= es[-1] - 1e-6  # the final state's energy is not below the sweep minimum
    g.close()


@pytest.mark.parametrize("name", ["cfg2_mid_sigma.json", "headline_mid_sigma.json"])
def test_middle_step_sigma_matches_the_oracle_golden(name):
    """L = 24, N = 12, D2h, D = 500 (the oracle-GPU parity configuration)
    and the headline L = 28, N = 12, D2h, D = 2500: sigma at the middle step
    on the same deterministic MPS (oracle.sadmrg.random_mps_at, rebuilt here)
    against the oracle's values stored by tests/golden/make_sigma_golden.py:
    512 sampled entries, the norm and a projection, within 1e-10 relative."""
    import json
    import os

    from paper_1312_2415_amd import SaDMRG
    from oracle import sadmrg as sd
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", name)))
    I = make_integrals(gold["L"], "D2h", gold["seed_integrals"])
    P = sd.Problem(I.h, I.eri, gold["N"], gold["twoS"], gold["irrep"], I.orb_irrep)
    dm = sd.random_mps_at(P, gold["D"], gold["seed_mps"], gold["step"])
    g = SaDMRG(gold["L"], 8, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(gold["N"], gold["twoS"], gold["irrep"])
    g.mps_import(sd.export_blob(dm))
    g.prepare_step()
    desc, n = g.psi_layout()
    assert n == gold["n"]
    assert [list(map(int, d[:5])) for d in desc] == gold["sectors"]
    x = np.random.default_rng(gold["x_seed"]).normal(size=n)
    got = g.sigma(x)
    g.close()
    scale = gold["max_abs_sigma"]
    assert np.abs(got[gold["index"]] - np.array(gold["value"])).max() <= 1e-10 * scale
    assert abs(np.linalg.norm(got) - gold["sigma_norm"]) <= 1e-10 * gold["sigma_norm"]
    r = np.random.default_rng(gold["r_seed"]).normal(size=n)
    assert abs(r @ got - gold["r_dot_sigma"]) <= 1e-10 * gold["sigma_norm"] * np.sqrt(n)
