"""The method-work counter (sadmrg_set_method_counter): the flops of the
sigma products with the structurally zero piece pairs of the enlarged
operator blocks skipped.  Checked against the same count made from the
oracle's enlarged blocks, where a piece pair is nonzero when its sub-block
holds a nonzero number (random integrals: no accidental zeros)."""
import numpy as np
import pytest

from oracle import sadmrg as sd
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu


def _pieces(E, m, dims, left):
    out = []
    for pc in E.pieces[m]:
        key = (m,) + pc
        size = dims[pc[0]] if left else dims[pc[1]]
        out.append((E.off[key], size))
    return out


def _shape(M, rp, cp):
    area, rows, cols = 0.0, np.zeros(M.shape[0], bool), np.zeros(M.shape[1], bool)
    for r0, rn in rp:
        for c0, cn in cp:
            if np.any(M[r0:r0 + rn, c0:c0 + cn] != 0.0):
                area += rn * cn
                rows[r0:r0 + rn] = True
                cols[c0:c0 + cn] = True
    return area, int(rows.sum()), int(cols.sum())


def _oracle_counts(P, dm, i):
    El, Er, Xe, Ye, secs = dm.enlarged(i)
    H = sd.Heff(P, Xe, Ye, secs)
    dx, dy = El.dim, Er.dim
    lp = {m: _pieces(El, m, El.sub, True) for m in secs}
    rp = {m: _pieces(Er, m, Er.sub, False) for m in secs}
    dense = method = 0.0
    for coef, Xo, Yo, hc in H.terms:
        if Yo is None:
            for (mb, mk), M in Xo.blocks.items():
                if mb in dx and mk in dx and mb == mk:
                    dense += 2.0 * M.shape[0] * M.shape[1] * dy[mk]
                    method += 2.0 * _shape(M, lp[mb], lp[mk])[0] * dy[mk]
            continue
        if Xo is None:
            for (mb, mk), M in Yo.blocks.items():
                if mb in dy and mk in dy and mb == mk:
                    dense += 2.0 * dx[mk] * M.shape[0] * M.shape[1]
                    method += 2.0 * dx[mk] * _shape(M, rp[mb], rp[mk])[0]
            continue
        for (mb, mk), A in Xo.blocks.items():
            if mb not in dx or mk not in dx or (mb, mk) not in Yo.blocks:
                continue
            Yb = Yo.blocks[(mb, mk)]
            R, K1, K2, C = dx[mb], dx[mk], dy[mk], dy[mb]
            nzA, rA, cA = _shape(A, lp[mb], lp[mk])
            nzY, rY, cY = _shape(Yb, rp[mb], rp[mk])
            dense += (2.0 if hc else 1.0) * min(2.0 * R * K2 * (K1 + C), 2.0 * K1 * C * (K2 + R))
            method += min(2.0 * nzA * K2 + 2.0 * rA * nzY, 2.0 * K1 * nzY + 2.0 * nzA * rY)
            if hc:
                method += min(2.0 * nzA * C + 2.0 * cA * nzY, 2.0 * R * nzY + 2.0 * nzA * cY)
    return dense, method


@pytest.mark.parametrize("case", [(8, 8, 0, "C1", 0, 24), (10, 8, 2, "D2h", 0, 40)])
def test_method_counter_matches_oracle_piece_structure(case):
    from paper_1312_2415_amd import SaDMRG
    L, N, twoS, group, irrep, D = case
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    g = SaDMRG(L, {"C1": 1, "D2h": 8}[group], I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, twoS, irrep)
    g.set_method_counter(True)
    ratios = []
    for i in range(L - 1):
        g.mps_import(sd.export_blob(dm))
        g.prepare_step()
        dense, method = _oracle_counts(P, dm, i)
        flops, _, _ = g.sigma_counters()
        step_method = g.stats_method()[2]
        print(f"step {i}: GPU performed {flops:.0f} method {step_method:.0f}; oracle dense {dense:.0f} "
              f"method {method:.0f}", flush=True)
        # the GPU performs every symmetry-allowed block (all-zero ones too), the
        # oracle keeps only blocks that received a contribution: the dense
        # counts may differ, the method counts skip zeros on both sides
        assert flops >= dense * (1 - 1e-12)
        assert abs(step_method - method) <= 1e-9 * method
        ratios.append(flops / step_method)
        if i < L - 2:
            dm.micro(i, D, "right")
    g.set_method_counter(False)
    g.close()
    print(f"performed / method flops per step: {np.round(ratios, 3)}")
    assert max(ratios) > 1.2
