"""Writes the oracle's sigma at the middle step of two configurations:

* cfg2_mid_sigma.json: L = 24, N = 12, singlet Ag, D2h (orbital irreps
  i mod 8), D_SU(2) = 500, integral seed 1002, step 11;
* headline_mid_sigma.json: L = 28, N = 12, singlet Ag, D2h, D_SU(2) = 2500,
  integral seed 1003 (the benchmark's problem), step 13.

The MPS is oracle.sadmrg.random_mps_at(P, D, seed=3, i=step): deterministic
random left- and right-normalised tensors with the centre on sites (i, i+1),
so that the same MPS can be rebuilt anywhere without optimisation.  Every
left and right block is built by the oracle (complementary operators,
renormalisation), then sigma = H_eff x for x ~ N(0, 1) from
numpy.random.default_rng(2024) over the step's flat layout.  Stored: the
layout, |sigma|, <r, sigma> for r from default_rng(2025), and 512 entries at
indices drawn from default_rng(2026).  Calls only oracle/ and synth/.

    python tests/golden/make_sigma_golden.py            (both, about 2 min)
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import sadmrg as sd  # noqa: E402
from synth.integrals import make_integrals  # noqa: E402

CONFIGS = {"cfg2_mid_sigma.json": (24, 12, 0, 0, 500, 1002, 3, 11),
           "headline_mid_sigma.json": (28, 12, 0, 0, 2500, 1003, 3, 13)}


def make(name, L, N, TWOS, IRREP, D, SEED_INT, SEED_MPS, STEP):
    t0 = time.time()
    I = make_integrals(L, "D2h", SEED_INT)
    P = sd.Problem(I.h, I.eri, N, TWOS, IRREP, I.orb_irrep)
    dm = sd.random_mps_at(P, D, SEED_MPS, STEP)
    dm.build_blocks_at(STEP)
    El, Er, Xe, Ye, secs = dm.enlarged(STEP)
    He = sd.Heff(P, Xe, Ye, secs)
    shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
    n = sum(a * b for a, b in shapes.values())
    x = np.random.default_rng(2024).normal(size=n)
    sig = sd.flatten(He.apply(sd.unflatten(x, shapes, secs)), secs)
    r = np.random.default_rng(2025).normal(size=n)
    idx = np.sort(np.random.default_rng(2026).choice(n, size=min(512, n), replace=False))
    out = {
        "workload": f"L={L} N={N} 2S={TWOS} irrep {IRREP} D2h, D_SU(2)={D}, integrals seed {SEED_INT}, "
                    f"random_mps_at(seed={SEED_MPS}, i={STEP})",
        "L": L, "N": N, "twoS": TWOS, "irrep": IRREP, "D": D, "seed_integrals": SEED_INT, "seed_mps": SEED_MPS,
        "step": STEP, "x_seed": 2024, "r_seed": 2025, "index_seed": 2026,
        "sectors": [[int(v) for v in list(m) + list(shapes[m])] for m in secs], "n": int(n),
        "sigma_norm": float(np.linalg.norm(sig)), "r_dot_sigma": float(r @ sig),
        "max_abs_sigma": float(np.abs(sig).max()),
        "index": [int(k) for k in idx], "value": [float(sig[k]) for k in idx],
        "oracle_seconds": time.time() - t0,
    }
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(out, f)
    print(f"{name}: n = {n}, |sigma| = {out['sigma_norm']:.12e}, {out['oracle_seconds']:.0f} s")


if __name__ == "__main__":
    for name, cfg in CONFIGS.items():
        if len(sys.argv) > 1 and name not in sys.argv[1:]:
            continue
        make(name, *cfg)
