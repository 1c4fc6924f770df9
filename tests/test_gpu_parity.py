"""GPU parity: libsadmrg (HIP, gfx950) against the CPU oracle.

Every GPU result is compared with the oracle on the same seeded inputs:
sigma vectors and the effective-Hamiltonian diagonal element by element
(relative 1e-10), and per-micro-iteration energies of whole sweeps (1e-8 E_h),
plus exactness against brute-force FCI where the bond dimension is complete.
"""
import copy

import numpy as np
import pytest

from oracle import sadmrg as sd
from oracle.fci import fci_solve
from synth.integrals import make_integrals

pytestmark = pytest.mark.gpu

ORDER = {"C1": 1, "C2": 2, "C2v": 4, "D2h": 8}


def _gpu(L, group, I):
    from paper_1312_2415_amd import SaDMRG
    g = SaDMRG(L, ORDER[group], I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    return g


@pytest.mark.parametrize("case", [(4, 4, 0, "C1", 0, 16), (5, 5, 1, "C2v", 1, 16), (6, 6, 2, "D2h", 0, 10),
                                  (6, 7, 1, "C2v", 3, 7), (8, 8, 0, "C1", 0, 40), (10, 10, 2, "D2h", 0, 30)])
def test_sigma_and_diagonal_match_oracle_at_every_step(case):
    L, N, twoS, group, irrep, D = case
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    for i in range(L - 1):
        print(f"case {case} step {i}", flush=True)
        g.mps_import(sd.export_blob(dm))
        g.prepare_step()
        desc, n = g.psi_layout()
        El, Er, Xe, Ye, secs = dm.enlarged(i)
        assert [tuple(d[:3]) for d in desc] == list(secs)
        He = sd.Heff(P, Xe, Ye, secs)
        shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
        x = np.random.default_rng(100 + i).normal(size=n)
        ref = sd.flatten(He.apply(sd.unflatten(x, shapes, secs)), secs)
        got = g.sigma(x)
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
        dref = sd.flatten(He.diagonal(shapes), secs)
        assert np.abs(g.heff_diagonal() - dref).max() <= 1e-10 * max(1.0, np.abs(dref).max())
        if i < L - 2:
            dm.micro(i, D, "right")
    g.close()


@pytest.mark.parametrize("case", [(8, 8, 0, "C1", 0, 64, 4, 1001), (6, 5, 1, "C2v", 1, 6, 2, 11),
                                  (10, 6, 2, "D2h", 0, 24, 2, 5), (12, 12, 0, "D2h", 0, 40, 1, 7)])
def test_sweep_energies_match_oracle(case):
    L, N, twoS, group, irrep, D, nsw, seed = case
    I = make_integrals(L, group, seed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    for _ in range(nsw):
        dm.sweep(D)
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    g.set_davidson(1e-9, 32, 200)
    g.mps_import(blob)
    for s in range(nsw):
        print(f"case {case} sweep {s}", flush=True)
        g.sweep(D)
    got, ref = g.trace(), np.array(dm.stats.energies)
    assert len(got) == len(ref)
    assert np.abs(got - ref).max() <= 1e-8
    assert abs(g.energy()[0] - dm.emin) <= 1e-8
    g.close()


def test_products_take_the_cheaper_contraction_order():
    """Each full product out[R x C] += c op(A)[R x K1] B[K1 x K2] op(C)[K2 x C]
    runs left first (2 R K2 (K1 + C) flops) or right first (2 K1 C (K2 + R)),
    whichever is cheaper: the flop counter equals the sum of the minima over
    the step's products, some steps do take the right-first order, and sigma
    stays on the oracle's (the per-step parity test above)."""
    L, N, twoS, group, irrep, D = 10, 8, 2, "D2h", 0, 30
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    g.mps_import(sd.export_blob(dm))
    saved = 0.0
    for i in range(L - 1):
        g.prepare_step()
        sh = g.task_shapes().astype(np.float64)
        R, K1, K2, C, fl = sh.T
        fl = fl.astype(int)
        ident_c, ident_a = (fl & 8) != 0, (fl & 4) != 0
        full = ~(ident_c | ident_a)
        left = 2 * R * K2 * (K1 + C)
        right = 2 * K1 * C * (K2 + R)
        want = (np.minimum(left, right)[full].sum() + (2 * R * K1 * C)[ident_c].sum()
                + (2 * R * K2 * C)[ident_a].sum())
        flops, _, ntasks = g.sigma_counters()
        assert ntasks == len(sh)
        assert abs(flops - want) <= 1e-9 * want
        saved += (left - np.minimum(left, right))[full].sum()
        if i < L - 2:
            g.advance(D, 1)
    assert saved > 0.0
    g.close()


def test_kept_enlargements_give_identical_sweeps():
    """Reusing the previous pass's enlarged blocks changes nothing: the
    traces with and without the cache agree bit for bit, also across a
    D change and an import that replaces every block."""
    L, N, twoS, group, irrep, D = 10, 8, 2, "D2h", 0, 30
    I = make_integrals(L, group, 41)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    runs = []
    for on in (True, False):
        g = _gpu(L, group, I)
        g.set_target(N, twoS, irrep)
        g.set_enlarge_cache(on)
        g.mps_import(blob)
        g.sweep(D)
        g.sweep(D + 10)
        g.mps_import(blob)
        g.sweep(D)
        runs.append(g.trace())
        g.close()
    assert np.array_equal(runs[0], runs[1])
    # the same energies as the oracle's first sweep from that state
    dm.sweep(D)
    n = 2 * (L - 1)
    assert np.abs(runs[0][-n:] - np.array(dm.stats.energies[:n])).max() <= 1e-8


def test_autotuned_launch_shape_keeps_sigma_and_sweeps():
    """The autotuner only changes how the products are spread over
    workgroups: sigma stays within rounding of the untuned one and of the
    oracle, and sweeps planned with the chosen shape match the oracle."""
    L, N, twoS, group, irrep, D = 10, 8, 0, "D2h", 0, 30
    I = make_integrals(L, group, 43)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    g.mps_import(blob)
    g.prepare_step()
    desc, n = g.psi_layout()
    x = np.random.default_rng(5).normal(size=n)
    y0 = g.sigma(x)
    (g1, g2), table = g.autotune(3)
    assert (g1, g2) in [t[0] for t in table]
    assert g1 in (0, 8) and g2 in (12, 16, 24, 32, 48, 64) and len(table) == 12
    assert all(ms > 0 for _, ms in table)
    y1 = g.sigma(x)
    assert np.abs(y1 - y0).max() <= 1e-12 * np.abs(y0).max()
    El, Er, Xe, Ye, secs = dm.enlarged(0)
    He = sd.Heff(P, Xe, Ye, secs)
    shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
    ref = sd.flatten(He.apply(sd.unflatten(x, shapes, secs)), secs)
    assert np.abs(y1 - ref).max() <= 1e-10 * np.abs(ref).max()
    g.mps_import(blob)
    g.sweep(D)
    dm.sweep(D)
    got, refe = g.trace(), np.array(dm.stats.energies)
    assert np.abs(got - refe).max() <= 1e-8
    g.close()


def test_fixed_launch_shape_and_device_memory_query():
    from paper_1312_2415_amd.binding import SadmrgError, device_memory
    L, N, twoS, group, irrep, D = 8, 6, 2, "C2v", 1, 24
    I = make_integrals(L, group, 44)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    blob = sd.export_blob(dm)
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    g.set_launch_shape(8, 48)
    for bad in ((-1, 12), (0, 65)):
        with pytest.raises(SadmrgError):
            g.set_launch_shape(*bad)
    g.mps_import(blob)
    g.sweep(D)
    dm.sweep(D)
    assert np.abs(g.trace() - np.array(dm.stats.energies)).max() <= 1e-8
    free, total = device_memory(0)
    assert 0 < free <= total
    g.close()


def test_config1_exact_at_fci_bond_dimension_with_own_initial_state():
    I = make_integrals(8, "C1", 1001)
    efci = fci_solve(I.h, I.eri, 8, 0)[0][0]
    g = _gpu(8, "C1", I)
    g.set_target(8, 0, 0)
    g.set_seed(7)
    e = g.solve([(128, 1e-10, 3)])
    assert abs(e - efci) <= 1e-9
    # variational below the FCI bond dimension
    g2 = _gpu(8, "C1", I)
    g2.set_target(8, 0, 0)
    e16 = g2.solve([(16, 1e-10, 3)])
    assert e16 >= efci - 1e-10
    assert g2.trace()[-1] > efci + 1e-6
    g.close()
    g2.close()


@pytest.mark.parametrize("N,twoS,group,irrep", [(6, 2, "C1", 0), (5, 1, "C2v", 1), (6, 0, "D2h", 0), (2, 0, "C1", 0),
                                                (12, 0, "C1", 0), (6, 6, "C1", 0), (11, 1, "C2v", 0)])
def test_spin_and_symmetry_targets_exact(N, twoS, group, irrep):
    # includes the one-hole and filled (N = 2L) limits and the fully polarised
    # sector (N < 2 is rejected: the one-body folding divides by N - 1)
    I = make_integrals(6, group, 21)
    efci = fci_solve(I.h, I.eri, N, twoS, irrep, I.orb_irrep)[0][0]
    g = _gpu(6, group, I)
    g.set_target(N, twoS, irrep)
    assert abs(g.solve([(64, 1e-11, 3)]) - efci) <= 1e-9
    g.close()


def test_discarded_weight_extrapolation_stages():
    """solve_extrapolated runs the scheme stage by stage: each stage's E(D)
    is the lowest energy of its last sweep and stays above FCI, E(D) does not
    rise with D, E0 is the least-squares intercept of the returned pairs, and
    a complete bond dimension (w = 0) returns the FCI energy itself."""
    I = make_integrals(8, "C1", 1001)
    efci = fci_solve(I.h, I.eri, 8, 0)[0][0]
    g = _gpu(8, "C1", I)
    g.set_target(8, 0, 0)
    g.set_seed(7)
    Ds = (28, 34, 40, 46)
    e0, c1, pts = g.solve_extrapolated([(D, 1e-10, 6) for D in Ds])
    assert [p[0] for p in pts] == list(Ds)
    es = np.array([p[2] for p in pts])
    ws = np.array([p[1] for p in pts])
    assert np.all(es >= efci - 1e-10) and np.all(ws > 0)
    assert np.all(np.diff(es) <= 1e-9)
    c1_ref, e0_ref = np.polyfit(ws, es, 1)
    assert abs(e0 - e0_ref) <= 1e-9 and abs(c1 - c1_ref) <= 1e-6 * max(1.0, abs(c1_ref))
    e0x, c1x, ptsx = g.solve_extrapolated([(128, 1e-10, 3)])
    assert ptsx[0][1] == 0.0 and c1x == 0.0
    assert abs(e0x - efci) <= 1e-9
    g.close()


def test_two_orbitals_single_step():
    # L = 2: the only micro-iteration covers the whole system (Hubbard dimer form)
    h = np.array([[0.0, -1.0], [-1.0, 0.0]])
    eri = np.zeros((2, 2, 2, 2))
    eri[0, 0, 0, 0] = eri[1, 1, 1, 1] = 4.0
    from paper_1312_2415_amd import SaDMRG
    g = SaDMRG(2, 1, [0, 0], device=0)
    g.set_integrals(h, eri)
    g.set_target(2, 0, 0)
    e = g.solve([(4, 1e-12, 2)])
    assert abs(e - (4.0 - np.sqrt(16.0 + 16.0)) / 2) < 1e-10
    g.close()


def test_mps_export_import_roundtrip():
    I = make_integrals(8, "C2", 9)
    g = _gpu(8, "C2", I)
    g.set_target(8, 2, 0)
    g.solve([(20, 1e-9, 1)])
    blob = g.mps_export()
    g2 = _gpu(8, "C2", I)
    g2.set_target(8, 2, 0)
    g2.mps_import(blob)
    assert g2.mps_export() == blob
    g2.prepare_step()
    desc, n = g2.psi_layout()
    x = np.random.default_rng(0).normal(size=n)
    y1 = g2.sigma(x)
    g.prepare_step()
    assert np.array_equal(y1, g.sigma(x))  # same operators, same task order: bitwise
    g.close()
    g2.close()


def test_rejects_bad_targets_and_integrals():
    from paper_1312_2415_amd.binding import SadmrgError
    I = make_integrals(4, "C1", 3)
    g = _gpu(4, "C1", I)
    with pytest.raises(SadmrgError):
        g.set_target(3, 0, 0)  # N - 2S odd
    with pytest.raises(SadmrgError):
        g.set_target(1, 1, 0)  # N < 2
    with pytest.raises(SadmrgError):
        g.set_target(0, 0, 0)  # empty
    with pytest.raises(SadmrgError):
        g.set_target(9, 1, 0)  # N > 2L
    with pytest.raises(SadmrgError):
        g.set_target(6, 4, 0)  # 2S beyond the 2L - N holes
    bad = I.eri.copy()
    bad[0, 1, 2, 3] += 1e-3
    with pytest.raises(SadmrgError):
        g.set_integrals(I.h, bad)
    g.close()


def test_sigma_matches_oracle_on_wide_blocks():
    """C1, L = 10, N = 10, D = 256: the enlarged sector blocks reach 144 wide,
    so products span several 64 x 64 output tiles in both directions, both
    GEMM passes run K beyond one 32-deep chunk, both contraction orders occur
    and the accumulating pass cuts tiles between workgroups (ordered partial
    reduction).  sigma and the diagonal against the oracle at every step."""
    L, N, twoS, group, irrep, D = 10, 10, 0, "C1", 0, 256
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    widest, orders, cuts = 0, set(), 0
    for i in range(L - 1):
        print(f"wide step {i}", flush=True)
        g.mps_import(sd.export_blob(dm))
        g.prepare_step()
        desc, n = g.psi_layout()
        El, Er, Xe, Ye, secs = dm.enlarged(i)
        assert [tuple(d[:3]) for d in desc] == list(secs)
        sh = g.task_shapes().astype(np.float64)
        R, K1, K2, C, fl = sh.T
        widest = max(widest, int(max(R.max(), K1.max(), K2.max(), C.max())))
        full = (fl.astype(int) & 12) == 0
        left, right = 2 * R * K2 * (K1 + C), 2 * K1 * C * (K2 + R)
        orders |= {"left"} if (left <= right)[full].any() else set()
        orders |= {"right"} if (right < left)[full].any() else set()
        cuts += g.plan_stats()[1][2]
        He = sd.Heff(P, Xe, Ye, secs)
        shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
        x = np.random.default_rng(300 + i).normal(size=n)
        ref = sd.flatten(He.apply(sd.unflatten(x, shapes, secs)), secs)
        got = g.sigma(x)
        assert np.abs(got - ref).max() <= 1e-10 * np.abs(ref).max()
        dref = sd.flatten(He.diagonal(shapes), secs)
        assert np.abs(g.heff_diagonal() - dref).max() <= 1e-10 * max(1.0, np.abs(dref).max())
        if i < L - 2:
            dm.micro(i, D, "right")
    g.close()
    assert widest > 128
    assert orders == {"left", "right"}
    assert cuts > 0


def test_xcd_order_gives_identical_sigma():
    """The XCD-grouped workgroup order only changes which workgroup runs
    which tile: sigma is bit for bit the same, and on the oracle's."""
    L, N, twoS, group, irrep, D = 10, 10, 0, "C1", 0, 120
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    for i in range(4):
        dm.micro(i, D, "right")
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    g.mps_import(sd.export_blob(dm))
    g.prepare_step()
    _, n = g.psi_layout()
    x = np.random.default_rng(5).normal(size=n)
    y0 = g.sigma(x)
    for p1, p2 in ((1, 0), (0, 1), (1, 1)):
        g.set_xcd_order(p1, p2)
        g.prepare_step()
        assert np.array_equal(g.sigma(x), y0)
    El, Er, Xe, Ye, secs = dm.enlarged(4)
    shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
    ref = sd.flatten(sd.Heff(P, Xe, Ye, secs).apply(sd.unflatten(x, shapes, secs)), secs)
    assert np.abs(y0 - ref).max() <= 1e-10 * np.abs(ref).max()
    g.close()



def test_traffic_order_keeps_sigma_on_the_oracle():
    """Contraction orders picked by the bytes a product streams
    (sadmrg_set_contraction_order(1)) instead of its flops: sigma stays on
    the oracle's at every step of the wide-block case, some products change
    order, and the flops never drop below the minimum-flop plan's."""
    L, N, twoS, group, irrep, D = 10, 10, 0, "C1", 0, 256
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    changed = 0.0
    for i in range(L - 1):
        print(f"traffic order step {i}", flush=True)
        g.mps_import(sd.export_blob(dm))
        g.set_contraction_order(0)
        g.prepare_step()
        f0 = g.sigma_counters()[0]
        g.set_contraction_order(1)
        g.prepare_step()
        f1 = g.sigma_counters()[0]
        assert f1 >= f0 * (1 - 1e-12)
        changed += f1 - f0
        desc, n = g.psi_layout()
        El, Er, Xe, Ye, secs = dm.enlarged(i)
        He = sd.Heff(P, Xe, Ye, secs)
        shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
        x = np.random.default_rng(700 + i).normal(size=n)
        ref = sd.flatten(He.apply(sd.unflatten(x, shapes, secs)), secs)
        assert np.abs(g.sigma(x) - ref).max() <= 1e-10 * np.abs(ref).max()
        if i < L - 2:
            dm.micro(i, D, "right")
    assert changed > 0.0
    from paper_1312_2415_amd.binding import SadmrgError
    with pytest.raises(SadmrgError):
        g.set_contraction_order(2)
    g.close()


def test_decomposition_of_wide_sectors_keeps_sweeps_on_the_oracle():
    """The wide-block case (C1, L = 10, D = 256: sector matrices with more than
    64 singular values, decomposed by block Jacobi): from the oracle's state
    at every step, two GPU micro-iterations against the oracle's two; the
    second one's energy depends on the first one's decomposition, truncation
    and renormalisation (1e-8 E_h), and the kept sector dimensions agree."""
    L, N, twoS, group, irrep, D = 10, 10, 0, "C1", 0, 256
    I = make_integrals(L, group, 11)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    g = _gpu(L, group, I)
    g.set_target(N, twoS, irrep)
    g.set_davidson(1e-9, 32, 200)
    widest = 0
    for i in range(L - 3):
        print(f"wide decomposition step {i}", flush=True)
        g.mps_import(sd.export_blob(dm))
        g.prepare_step()
        desc, _ = g.psi_layout()
        widest = max(widest, int(np.minimum(desc[:, 3], desc[:, 4]).max()))
        e_gpu = [g.advance(D, 1)]
        g.prepare_step()
        desc1, _ = g.psi_layout()
        e_gpu.append(g.advance(D, 1))
        e_ora = [dm.micro(i, D, "right")]
        after = copy.deepcopy(dm)  # the start of step i + 1
        El, Er, _, _, secs = dm.enlarged(i + 1)
        assert sorted((int(r[3]), int(r[4])) for r in desc1) == sorted((El.dim[m], Er.dim[m]) for m in secs)
        e_ora.append(dm.micro(i + 1, D, "right"))
        assert abs(e_gpu[0] - e_ora[0]) <= 1e-8
        assert abs(e_gpu[1] - e_ora[1]) <= 1e-8
        dm = after
    assert widest >= 64
    g.close()
