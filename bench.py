#!/usr/bin/env python3
"""Benchmark: spin-adapted two-site DMRG sweeps on one MI355X.

Workload (the headline configuration): L = 28 orbitals, N = 12 electrons,
singlet, D2h with round-robin orbital irreps, target irrep Ag, reduced bond
dimension D = 2500, seeded synthetic integrals (stand-in for the paper's
carbon-dimer cc-pVDZ integrals, which are not available).

A "step" is one macro-iteration (a left-to-right plus a right-to-left pass;
every micro-iteration: enlargement and complementary operators, Davidson with
the H_eff sigma product, SVD truncation, renormalisation).  The MPS starts
random at bond dimension D and every sweep (warm-up and timed) runs at D, so
every kernel launch of the run has the shapes of the headline workload.

Reported `value` is the sigma-product rate of the plain FP64 path: algorithmic
FP64 flops of all H_eff*psi calls in the timed sweeps (every block triple
product in the cheaper of its two contraction orders, the order the kernels
run) divided by their kernel time (HIP events on the library stream).  `ms_per_step` is the wall time per
FP64 sweep.  `mixed` and `mixed_bf16x3` repeat the timed sweeps from the same
state with FP32 / BF16x3 sigma products in Davidson (one FP64 Davidson step
per micro-iteration gives the energy) and report s/sweep, speedup, the reduced
sigma rate and its roofline fraction, and |dE| and RDM errors against the FP64
sweeps.  `batch` sweeps 64 independent small problems in lockstep against the
same sweeps one after another.  `roots` sweeps one GPU's share of twelve roots
of the headline problem (S in {0, 1, 2} times four irreps, in separate
symmetry sectors, dealt round-robin to GPUs) in lockstep, in FP64 and in mixed
precision from the same states, with per-root |dE| and RDM errors.  `grad`
is the energy adjoint (spin-summed 1- and 2-RDM as dE/dh and dE/d(ij|kl)) at
L = 36, D = 2500, checked by central differences of the frozen-MPS energy
along a few integral orbits.  `autotune` records the launch-shape choice.  `roofline`
describes the dominant sigma kernel (the grouped-GEMM pass with the larger
share of sigma time): its algorithmic flops per launch over its mean launch
duration, against the FP64 MFMA peak.  `traffic` is filled from the committed
HBM-counter summary when that summary was taken on the current kernel source.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "H_eff·ψ TFLOP/s + s/sweep, FP64 vs mixed at |ΔE|≤1e-6 Eh, L=28 D=2500"
FP64_MFMA_PEAK = 78.6  # TFLOP/s, MI355X dense FP64 matrix peak
FP32_MFMA_PEAK = 157.3  # TFLOP/s, dense FP32 matrix peak
BF16_MFMA_PEAK = 2500.0  # TFLOP/s, dense BF16 matrix peak (a BF16x3 product costs three)
HBM_PEAK = 8000.0  # GB/s
KERNEL_SRC = os.path.join(ROOT, "paper_1312_2415_amd", "csrc", "kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gemm_kernel_sigma_L28_N12_D2500_traffic.json")
PASS_KERNEL = {"pass1": "gemm_tile_kernel<double, 0> (sigma pass 1: T = X psi or U = psi Y^T per product)",
               "pass2": "gemm_stream_kernel<double, 1> (sigma pass 2: sigma += T Y^T or X U)"}


def kernel_source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def stored_traffic(pass_name: str):
    """HBM bytes per launch of a sigma pass from the committed counter summary,
    or None when it is missing or was taken on other kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernels_hip_sha256") != kernel_source_hash():
        return None
    ent = rec.get("per_launch", {}).get(pass_name)
    if not ent:
        return None
    return ent.get("fetch_bytes", 0.0) + ent.get("write_bytes", 0.0)


def sigma_flops_oracle(H):
    """Flops of the oracle's H_eff application counted as the GPU path counts
    them: dense enlarged-block triple products, each in the cheaper of its
    two contraction orders (the oracle's own blocks are dense as well)."""
    f = 0.0
    for coef, Xo, Yo, hc in H.terms:
        mult = 2.0 if hc else 1.0
        if Yo is None:
            for (mb, mk), M in Xo.blocks.items():
                if mb in H.dy and mk in H.dy:
                    f += 2.0 * M.shape[0] * M.shape[1] * H.dy[mk]
            continue
        if Xo is None:
            for (mb, mk), M in Yo.blocks.items():
                if mb in H.dx and mk in H.dx:
                    f += 2.0 * H.dx[mk] * M.shape[1] * M.shape[0]
            continue
        for (mb, mk), MX in Xo.blocks.items():
            if mb not in H.dy or mk not in H.dy or (mb, mk) not in Yo.blocks:
                continue
            R, K1, K2, C = H.dx[mb], H.dx[mk], H.dy[mk], H.dy[mb]
            f += mult * min(2.0 * R * K2 * (K1 + C), 2.0 * K1 * C * (K2 + R))
    return f


def physical_cores():
    """Physical cores of the host (lscpu), or None."""
    import subprocess
    try:
        out = subprocess.run(["lscpu", "-p=CORE,SOCKET"], capture_output=True, text=True, timeout=10).stdout
        return len({line for line in out.splitlines() if line and not line.startswith("#")}) or None
    except Exception:
        return None


def cpu_baseline(seconds: float, L: int, N: int, twoS: int, irrep: int, seed: int, D: int, step: int):
    """The oracle and the GPU on the same sigma product: the middle step of
    the headline shape (L orbitals, N electrons, D_SU(2) = D, D2h, the same
    integrals), on the deterministic MPS oracle.sadmrg.random_mps_at(P, D, 3,
    step) that both sides build (random left- and right-normalised tensors,
    equal split of D over the sectors).  The oracle builds every block of the
    chain (not timed), then applies H_eff until `seconds` of sigma time with
    all of its BLAS threads, and once more on one thread; the GPU imports the
    same MPS and times its sigma on the same step.  Flops: the GPU path's
    definition, counted from the oracle's blocks."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import sadmrg as sd
    from paper_1312_2415_amd import SaDMRG
    from synth.integrals import make_integrals

    I = make_integrals(L, "D2h", seed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    t0 = time.perf_counter()
    dm = sd.random_mps_at(P, D, 3, step)
    dm.build_blocks_at(step)
    El, Er, Xe, Ye, secs = dm.enlarged(step)
    H = sd.Heff(P, Xe, Ye, secs)
    shapes = {m: (El.dim[m], Er.dim[m]) for m in secs}
    H.dx = {m: shapes[m][0] for m in secs}
    H.dy = {m: shapes[m][1] for m in secs}
    flops = sigma_flops_oracle(H)
    t_setup = time.perf_counter() - t0
    n = sum(a * b for a, b in shapes.values())
    x = np.random.default_rng(7).normal(size=n)
    psi = sd.unflatten(x, shapes, secs)
    print(f"cpu baseline: oracle blocks of L={L} D={D} step {step} built in {t_setup:.0f}s, |psi| = {n}, "
          f"{flops:.3e} flop per sigma", file=sys.stderr, flush=True)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    calls, t_all = 0, 0.0
    while calls < 1 or t_all < seconds:
        t = time.perf_counter()
        y_ref = sd.flatten(H.apply(psi), secs)
        t_all += time.perf_counter() - t
        calls += 1
    with threadpool_limits(limits=1):
        t = time.perf_counter()
        H.apply(psi)
        t_one = time.perf_counter() - t
    print(f"cpu baseline: {t_all / calls:.2f}s per sigma on {threads} threads, {t_one:.2f}s on one",
          file=sys.stderr, flush=True)
    g = SaDMRG(L, 8, I.orb_irrep, device=0)
    try:
        g.set_integrals(I.h, I.eri)
        g.set_target(N, twoS, irrep)
        g.mps_import(sd.export_blob(dm))
        g.prepare_step()
        y = g.sigma(x)
        err = float(np.abs(y - y_ref).max() / np.abs(y_ref).max())
        gflops, _, _ = g.sigma_counters()
        g.stats_reset()
        for _ in range(10):  # kernel time from the library's HIP events (host copies outside)
            g.sigma(x)
        st = g.stats()
        t_gpu = st["t_sigma"] / max(st["n_sigma"], 1)
    finally:
        g.close()
    rate = flops / (t_all / calls) / 1e12
    return {"value": rate, "unit": "TFLOP/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle sigma at the middle step (i={step}) of L={L} N={N} 2S={twoS} D2h D_SU(2)={D} "
                      f"on oracle.sadmrg.random_mps_at(seed 3): {calls} call(s), {t_all:.1f}s of sigma time on "
                      f"{threads} BLAS threads (block building {t_setup:.0f}s, not timed) and one call on one "
                      f"thread; flops counted as for the GPU path",
            "oracle_seconds_per_sigma": t_all / calls, "oracle_seconds_per_sigma_one_thread": t_one,
            "oracle_tflops_one_thread": flops / t_one / 1e12, "physical_cores": physical_cores(),
            "flops_per_sigma": flops, "gpu_flops_per_sigma": gflops, "psi_length": n,
            "gpu_ms_per_sigma_same_step": 1e3 * t_gpu, "gpu_speedup_same_step": (t_all / calls) / t_gpu,
            "gpu_vs_oracle_sigma_max_rel_diff": err}


def batch_workload(n, seed):
    """Independent small problems of mixed size: L uniform in 10..20, N = L/2
    rounded to an even number, S in {0, 1}, D uniform in 128..1024, D2h with
    orbital irreps round-robin, target Ag, each with its own integral seed."""
    rng = np.random.default_rng(seed)
    specs = []
    for k in range(n):
        L = int(rng.integers(10, 21))
        specs.append({"L": L, "N": 2 * int(round(L / 4)), "twoS": 2 * int(rng.integers(0, 2)),
                      "D": int(rng.integers(128, 1025)), "seed": seed * 1000 + k})
    return specs


def batch_bench(n, seed, prec, mixed_tol, graph=4):
    """One lockstep sweep of n problems (sadmrg_batch_sweep) against the same
    problems swept one after another from the same states, and (graph > 0)
    the same lockstep sweep again with the Davidson iterations replayed from
    a recorded HIP graph, `graph` replays per host check."""
    from paper_1312_2415_amd import SaDMRG
    from paper_1312_2415_amd.binding import batch_sweep
    from synth.integrals import make_integrals
    specs = batch_workload(n, seed)
    t0 = time.perf_counter()
    gs = []
    for sp in specs:
        I = make_integrals(sp["L"], "D2h", sp["seed"])
        g = SaDMRG(sp["L"], 8, I.orb_irrep, device=0)
        g.set_integrals(I.h, I.eri)
        g.set_target(sp["N"], sp["twoS"], 0)
        g.set_seed(sp["seed"])
        g.set_davidson(1e-7, 32, 100)
        g.set_precision(prec, mixed_tol)
        g.init_mps(sp["D"])
        gs.append(g)
    Ds = [sp["D"] for sp in specs]
    t_init = time.perf_counter() - t0
    t0 = time.perf_counter()
    batch_sweep(gs, Ds)  # warm-up: pools, kept enlargements, a converging state
    t_warm = time.perf_counter() - t0
    print(f"batch of {n}: init {t_init:.1f}s, warm-up lockstep sweep {t_warm:.1f}s", file=sys.stderr, flush=True)
    blobs = [g.mps_export() for g in gs]
    t0 = time.perf_counter()
    eb, st, _ = batch_sweep(gs, Ds)
    t_batch = time.perf_counter() - t0
    print(f"batch of {n}: lockstep sweep {t_batch:.2f}s", file=sys.stderr, flush=True)
    rec = None
    if graph > 0:
        for g, b in zip(gs, blobs):
            g.mps_import(b)
            g.set_davidson_graph(graph)
            g.stats_reset()
        t0 = time.perf_counter()
        eg, stg, _ = batch_sweep(gs, Ds)
        t_graph = time.perf_counter() - t0
        sg = [g.stats_graph() for g in gs]
        rec = {"replays_per_host_check": graph, "s_per_lockstep_sweep": t_graph,
               "speedup_vs_host_driven_lockstep": t_batch / t_graph,
               "speedup_vs_separate_sweeps": None,
               "recordings": int(sum(x["records"] for x in sg)),
               "replayed_segment_seconds": float(sum(x["seconds"] for x in sg)),
               "recording_host_seconds": float(sum(x["record_seconds"] for x in sg)),
               "sigma_products_in_replays": int(sum(x["sigma_calls"] for x in sg)),
               "host_phase_wall_seconds": stg["wall"],
               "max_abs_dE_vs_host_driven_lockstep": float(max(abs(a - b) for a, b in zip(eg, eb)))}
        print(f"batch of {n}: lockstep sweep with recorded Davidson iterations {t_graph:.2f}s", file=sys.stderr,
              flush=True)
        for g in gs:
            g.set_davidson_graph(0)
    for g, b in zip(gs, blobs):
        g.mps_import(b)
    t0 = time.perf_counter()
    es = [g.sweep(D)[0] for g, D in zip(gs, Ds)]
    t_sep = time.perf_counter() - t0
    print(f"batch of {n}: separate sweeps {t_sep:.2f}s", file=sys.stderr, flush=True)
    for g in gs:
        g.close()
    t_sh = st["t_sigma"] + st["t_sigma32"]
    f_sh = st["flops_sigma"] + st["flops_sigma32"]
    if rec is not None:
        rec["speedup_vs_separate_sweeps"] = t_sep / rec["s_per_lockstep_sweep"]
    return {
        "workload": "independent problems, L uniform 10..20, N = L/2 rounded to even, S in {0,1}, "
                    "D_SU(2) uniform 128..1024, D2h round-robin orbital irreps, own integral seed each",
        "instances": n, "seed": seed,
        "precision": "FP32 sigma in Davidson + one FP64 Davidson step per micro-iteration" if prec == 1 else "FP64",
        "s_per_lockstep_sweep": t_batch,
        "s_per_separate_sweeps": t_sep,
        "speedup": t_sep / t_batch,
        "shared_sigma_launch_seconds": t_sh,
        "shared_sigma_tflops": f_sh / max(t_sh, 1e-12) / 1e12,
        "shared_sigma_launches": st["n_sigma"] + st["n_sigma32"],
        "host_phase_wall_seconds": st["wall"],
        "max_abs_dE_lockstep_vs_separate": float(max(abs(a - b) for a, b in zip(eb, es))),
        "recorded_davidson": rec,
        "L": [sp["L"] for sp in specs], "D": Ds,
    }


ROOT_TARGETS = [(2 * s, ir) for s in (0, 1, 2) for ir in (0, 1, 2, 3)]  # (2S, irrep) of the twelve roots


def roots_bench(group, L, N, D, seed, warm, dav_tol, mixed_tol, refine=1, refine_tol=0.0):
    """All twelve roots of the headline problem, in separate (S, irrep)
    sectors (S in {0, 1, 2} times four irreps), swept on one GPU in
    sequential lockstep groups of `group` (sadmrg_batch_sweep; a group fills
    most of the 288 GB).  Per group: `warm` FP64 lockstep sweeps from random
    MPS, one timed FP64 lockstep sweep, then from the same states one timed
    FP32 and one timed BF16x3 lockstep sweep (FP64 refinement), with per-root
    |dE| and RDM errors against the FP64 sweep; the first group also sweeps
    its roots one after another in FP64 for the lockstep speedup."""
    from paper_1312_2415_amd import SaDMRG
    from paper_1312_2415_amd.binding import batch_sweep, device_memory
    from synth.integrals import make_integrals
    if group < 1 or 12 % group:
        raise ValueError("roots: the group size must divide 12")
    I = make_integrals(L, "D2h", seed)
    per, t64s, t32s, tb3s, fl64, tt64, fl32, tt32, flb3, ttb3 = [], [], [], [], 0, 0, 0, 0, 0, 0
    tsep = t64_first = None
    mem_used = 0.0
    for g0 in range(0, 12, group):
        targets = ROOT_TARGETS[g0:g0 + group]
        gs = []
        try:
            for j, (twoS, irrep) in enumerate(targets):
                g = SaDMRG(L, 8, I.orb_irrep, device=0)
                gs.append(g)
                g.set_integrals(I.h, I.eri)
                g.set_target(N, twoS, irrep)
                g.set_seed(seed + 17 * (g0 + j))
                g.set_davidson(dav_tol, 32, 100)
                g.init_mps(D)
            for w in range(warm):
                t = time.perf_counter()
                batch_sweep(gs, D)
                print(f"roots {targets}: warm-up lockstep sweep {w + 1}/{warm} {time.perf_counter() - t:.1f}s",
                      file=sys.stderr, flush=True)
            blobs = [g.mps_export() for g in gs]
            n0 = [len(g.trace()) for g in gs]
            t = time.perf_counter()
            e64, st64, _ = batch_sweep(gs, D)
            t64 = time.perf_counter() - t
            free, total = device_memory(0)
            mem_used = max(mem_used, (total - free) / 2**30)
            tr64 = [np.array(g.trace()[n:]) for g, n in zip(gs, n0)]
            r64 = [g.rdm() for g in gs]
            print(f"roots {targets}: FP64 lockstep sweep {t64:.2f}s", file=sys.stderr, flush=True)
            t64s.append(t64)
            fl64 += st64["flops_sigma"]
            tt64 += st64["t_sigma"]
            if g0 == 0:
                t = time.perf_counter()
                for g, b in zip(gs, blobs):
                    g.mps_import(b)
                    g.sweep(D)
                tsep = time.perf_counter() - t
                t64_first = t64
                print(f"roots {targets}: separate FP64 sweeps {tsep:.2f}s", file=sys.stderr, flush=True)
            res = {}
            for mode in (1, 2):
                n1 = []
                for g, b in zip(gs, blobs):
                    g.set_precision(mode, mixed_tol)
                    g.set_refinement(refine)
                    g.set_refinement_tol(refine_tol)
                    g.mps_import(b)
                    n1.append(len(g.trace()))
                t = time.perf_counter()
                em, stm, _ = batch_sweep(gs, D)
                tm = time.perf_counter() - t
                trm = [np.array(g.trace()[n:]) for g, n in zip(gs, n1)]
                rm = [g.rdm() for g in gs]
                res[mode] = (em, trm, rm, tm)
                print(f"roots {targets}: {'FP32' if mode == 1 else 'BF16x3'} lockstep sweep {tm:.2f}s",
                      file=sys.stderr, flush=True)
                if mode == 1:
                    t32s.append(tm)
                    fl32 += stm["flops_sigma32"]
                    tt32 += stm["t_sigma32"]
                else:
                    tb3s.append(tm)
                    flb3 += stm["flops_sigma32"]
                    ttb3 += stm["t_sigma32"]
            for j, (twoS, irrep) in enumerate(targets):
                rec = {"twoS": twoS, "irrep": irrep, "energy_fp64": e64[j]}
                for mode, key in ((1, "fp32"), (2, "bf16x3")):
                    em, trm, rm, _ = res[mode]
                    same = len(trm[j]) == len(tr64[j]) and len(tr64[j]) > 0
                    rec[key] = {"energy": em[j], "abs_dE": abs(em[j] - e64[j]),
                                "max_abs_dE_per_micro_iteration":
                                    float(np.abs(trm[j] - tr64[j]).max()) if same else None,
                                "rdm_max_abs_error": {"gamma": float(np.abs(rm[j][0] - r64[j][0]).max()),
                                                      "Gamma": float(np.abs(rm[j][1] - r64[j][1]).max())}}
                per.append(rec)
        finally:
            for g in gs:
                g.close()

    def worst(key, f):
        return max(f(r[key]) for r in per)

    out = {
        "workload": f"the twelve roots of L={L} N={N} D2h D_SU(2)={D} (seed {seed}): (2S, irrep) in "
                    f"{[list(t) for t in ROOT_TARGETS]}, one GPU, lockstep groups of {group}",
        "roots": 12, "group": group, "warmup_lockstep_sweeps": warm, "fp64_refinement_steps": refine,
        "fp64_refinement_residual_target": refine_tol,
        "s_per_lockstep_sweep_fp64": t64s, "s_per_lockstep_sweep_fp32": t32s,
        "s_per_lockstep_sweep_bf16x3": tb3s,
        "s_all_twelve_fp64": sum(t64s), "s_all_twelve_fp32": sum(t32s), "s_all_twelve_bf16x3": sum(tb3s),
        "speedup_fp32_vs_fp64": sum(t64s) / sum(t32s), "speedup_bf16x3_vs_fp64": sum(t64s) / sum(tb3s),
        "first_group_s_separate_fp64": tsep, "first_group_lockstep_speedup_fp64": tsep / t64_first,
        "sigma_tflops_fp64": fl64 / max(tt64, 1e-12) / 1e12,
        "sigma_tflops_fp32": fl32 / max(tt32, 1e-12) / 1e12,
        "sigma_tflops_bf16x3": flb3 / max(ttb3, 1e-12) / 1e12,
        "device_memory_used_GiB": mem_used,
        "max_abs_dE": {"fp32": worst("fp32", lambda r: r["abs_dE"]), "bf16x3": worst("bf16x3", lambda r: r["abs_dE"])},
        "max_rdm_abs_error": {k: worst(k, lambda r: max(r["rdm_max_abs_error"].values()))
                              for k in ("fp32", "bf16x3")},
        "per_root": per,
    }
    out["target_met"] = {k: bool(out["max_abs_dE"][k] <= 1e-6 and out["max_rdm_abs_error"][k] <= 1e-5)
                         for k in ("fp32", "bf16x3")}
    return out


def grad_bench(L, N, D, seed, warm, n_orbits, tau, n_dir=200, ckpt=6):
    """Energy adjoint at the differentiation configuration (L orbitals, N
    electrons, singlet Ag, D2h): the spin-summed 1- and 2-RDM of the MPS after
    `warm` sweeps at D, as dE/dh and dE/d(ij|kl), against central differences
    of E = <psi|H|psi> for that same frozen MPS along symmetry-allowed integral
    orbits (every evaluation rebuilds all renormalised operators from the MPS
    with the shifted integrals), and along one direction that moves `n_dir`
    random symmetry-allowed entries (with their symmetry partners) at once.
    At fixed psi, E is linear in the integrals, so the difference quotient is
    exact up to rounding."""
    from paper_1312_2415_amd import SaDMRG
    from synth.integrals import make_integrals
    I = make_integrals(L, "D2h", seed)
    irr = np.asarray(I.orb_irrep)
    g = SaDMRG(L, 8, irr, device=0)
    try:
        g.set_integrals(I.h, I.eri)
        g.set_target(N, 0, 0)
        g.set_davidson(1e-7, 32, 100)
        t = time.perf_counter()
        g.init_mps(D)
        for w in range(warm):
            ts = time.perf_counter()
            e, _ = g.sweep(D)
            print(f"grad: sweep {w + 1}/{warm} L={L} D={D} E={e:.10f} {time.perf_counter() - ts:.1f}s",
                  file=sys.stderr, flush=True)
        t_sweeps = time.perf_counter() - t
        blob = g.mps_export()
        t = time.perf_counter()
        g1, g2, e0 = g.rdm()
        t_rdm = time.perf_counter() - t
        e_id = I.e_const + float(np.einsum("pq,pq", I.h, g1)) + 0.5 * float(np.einsum("ikjl,ijkl", I.eri, g2))
        dv_of = g2.transpose(0, 2, 1, 3)  # dE/d(ik|jl) = Gamma[i,j,k,l] / 2 at [i,k,j,l]
        rng = np.random.default_rng(seed + 5)
        rows = []
        t_fd = time.perf_counter()
        for k in range(n_orbits):
            dh = np.zeros((L, L))
            dv = np.zeros((L,) * 4)
            if k % 2 == 0:  # one-body entry h_pq = h_qp of one irrep
                while True:
                    p, q = (int(x) for x in rng.integers(0, L, 2))
                    if irr[p] == irr[q]:
                        break
                dh[p, q] = dh[q, p] = 1.0
                label = f"h[{p},{q}]"
            else:  # the eightfold orbit of one allowed (ij|kl)
                while True:
                    i, j, kk, l = (int(x) for x in rng.integers(0, L, 4))
                    if irr[i] ^ irr[j] ^ irr[kk] ^ irr[l] == 0:
                        break
                for a, b, c, d in ((i, j, kk, l), (j, i, kk, l), (i, j, l, kk), (j, i, l, kk),
                                   (kk, l, i, j), (l, kk, i, j), (kk, l, j, i), (l, kk, j, i)):
                    dv[a, b, c, d] = 1.0
                label = f"({i}{j}|{kk}{l})"
            pred = float(np.sum(g1 * dh)) + 0.5 * float(np.sum(dv_of * dv))
            es = []
            for sgn in (1.0, -1.0):
                g.set_integrals(I.h + sgn * tau * dh, I.eri + sgn * tau * dv)
                g.mps_import(blob)
                es.append(g.rdm(two_body=False)[2])
            fd = (es[0] - es[1]) / (2.0 * tau)
            rows.append({"entry": label, "adjoint": pred, "finite_difference": fd, "abs_diff": abs(fd - pred)})
            print(f"grad: {label} adjoint {pred:.10f} fd {fd:.10f}", file=sys.stderr, flush=True)
        # one direction that moves n_dir random symmetry-allowed entries at
        # once (each with its symmetry partners, random weights): the
        # adjoint's contraction with it against one central difference
        dh = np.zeros((L, L))
        dv = np.zeros((L,) * 4)
        picked = 0
        while picked < n_dir:
            w = float(rng.normal())
            if rng.random() < 0.1:
                p, q = (int(x) for x in rng.integers(0, L, 2))
                if irr[p] != irr[q]:
                    continue
                dh[p, q] += w
                if p != q:
                    dh[q, p] += w
            else:
                i, j, kk, l = (int(x) for x in rng.integers(0, L, 4))
                if irr[i] ^ irr[j] ^ irr[kk] ^ irr[l]:
                    continue
                for a, b, c, d in {(i, j, kk, l), (j, i, kk, l), (i, j, l, kk), (j, i, l, kk),
                                   (kk, l, i, j), (l, kk, i, j), (kk, l, j, i), (l, kk, j, i)}:
                    dv[a, b, c, d] += w
            picked += 1
        pred_dir = float(np.sum(g1 * dh)) + 0.5 * float(np.sum(dv_of * dv))
        es = []
        for sgn in (1.0, -1.0):
            g.set_integrals(I.h + sgn * tau * dh, I.eri + sgn * tau * dv)
            g.mps_import(blob)
            es.append(g.rdm(two_body=False)[2])
        fd_dir = (es[0] - es[1]) / (2.0 * tau)
        print(f"grad: direction over {n_dir} entries: adjoint {pred_dir:.10f} fd {fd_dir:.10f}", file=sys.stderr,
              flush=True)
        t_fd = time.perf_counter() - t_fd
        # the adjoint again with renormalised operators recomputed instead of
        # stored (blocks kept every `ckpt` bonds), on the original integrals
        ck = None
        if ckpt > 0:
            full_blocks = g.stats_blocks()
            g.set_integrals(I.h, I.eri)
            g.set_block_checkpoints(ckpt)
            g.stats_reset()
            t = time.perf_counter()
            g.mps_import(blob)
            t_imp = time.perf_counter() - t
            t = time.perf_counter()
            c1, c2, ec = g.rdm()
            t_ck = time.perf_counter() - t
            sb = g.stats_blocks()
            ck = {"interval": ckpt, "seconds_import": t_imp, "seconds_rdm": t_ck,
                  "block_bytes_max": sb["max_bytes"], "block_bytes_max_all_stored": full_blocks["max_bytes"],
                  "blocks_rebuilt_in_rdm": sb["rebuilt"], "rebuild_seconds": sb["seconds"],
                  "max_abs_diff_gamma": float(np.abs(c1 - g1).max()),
                  "max_abs_diff_Gamma": float(np.abs(c2 - g2).max()), "abs_diff_energy": abs(ec - e0)}
            print(f"grad: checkpoints every {ckpt} bonds: rdm {t_ck:.1f}s, block bytes "
                  f"{sb['max_bytes'] / 2**30:.1f} GiB against {full_blocks['max_bytes'] / 2**30:.1f} GiB, "
                  f"|dGamma| {ck['max_abs_diff_Gamma']:.1e}", file=sys.stderr, flush=True)
        return {
            "operator_recomputation": ck,
            "fd_direction": {"entries": n_dir, "adjoint": pred_dir, "finite_difference": fd_dir,
                             "abs_diff": abs(fd_dir - pred_dir),
                             "rel_diff": abs(fd_dir - pred_dir) / max(abs(pred_dir), 1e-300)},
            "workload": f"energy adjoint at L={L} N={N} 2S=0 D2h irrep Ag D_SU(2)={D}, seeded synthetic integrals "
                        f"(seed {seed}), MPS after {warm} sweeps from random",
            "seconds_sweeps": t_sweeps, "seconds_rdm": t_rdm, "energy": e0,
            "energy_identity_error": abs(e_id - e0), "trace_gamma": float(np.trace(g1)),
            "fd_step": tau, "fd_orbits": n_orbits, "fd_seconds_per_evaluation": t_fd / max(2 * n_orbits, 1),
            "max_abs_diff": max((r["abs_diff"] for r in rows), default=None),
            "fd": rows,
        }
    finally:
        g.close()


def dmrgscf_bench(L, N, D, seed, n_core, max_iter, sweeps, dav_tol):
    """DMRG-SCF (section "DMRG-SCF", sadmrg_dmrgscf) on the differentiation
    configuration's integrals: the first n_core orbitals doubly occupied and
    optimised, the other L - n_core active with N - 2 n_core electrons (the
    paper's DMRG-SCF(34o, 8e) partition of 36 orbitals), D_SU(2) = D;
    `max_iter` augmented-Hessian iterations, each after `sweeps` sweeps from
    the previous MPS."""
    from paper_1312_2415_amd import SaDMRG
    from synth.integrals import make_integrals
    I = make_integrals(L, "D2h", seed)
    cls = [0] * n_core + [1] * (L - n_core)
    act = list(range(n_core, L))
    g = SaDMRG(L - n_core, 8, np.asarray(I.orb_irrep)[act], device=0)
    try:
        g.set_target(N - 2 * n_core, 0, 0)
        g.set_davidson(dav_tol, 32, 100)
        t = time.perf_counter()
        e, U, hist, it = g.dmrgscf(I.orb_irrep, cls, I.h, I.eri, [(D, 1e-8, sweeps)], grad_tol=1e-6,
                                   max_iter=max_iter)
        t = time.perf_counter() - t
    finally:
        g.close()
    for k, (ek, gk) in enumerate(hist):
        print(f"dmrgscf: iteration {k}: E {ek:.10f} |g| {gk:.3e}", file=sys.stderr, flush=True)
    return {"workload": f"DMRG-SCF, L={L} orbitals ({n_core} core, {L - n_core} active, {N - 2 * n_core} active "
                        f"electrons), singlet Ag, D2h, D_SU(2)={D}, seeded synthetic integrals (seed {seed}), "
                        f"{sweeps} sweep(s) per iteration",
            "iterations": it, "seconds": t, "seconds_per_iteration": t / max(it, 1), "energy": e,
            "history": [{"energy": ek, "gradient_norm": gk} for ek, gk in hist],
            "orbital_orthonormality_error": float(np.abs(U.T @ U - np.eye(L)).max())}


TABLE1 = [(200, 1e-8, 2, 0.03), (200, 1e-8, 3, 0.0), (500, 1e-8, 2, 0.03), (500, 1e-8, 5, 0.0),
          (1000, 1e-8, 2, 0.03), (1000, 1e-8, 5, 0.0), (1500, 1e-8, 2, 0.03), (1500, 1e-8, 5, 0.0),
          (2000, 1e-8, 2, 0.03), (2000, 1e-8, 5, 0.0), (2500, 1e-8, 2, 0.03), (2500, 1e-8, 12, 0.0)]


def scheme_bench(L, N, twoS, irrep, seed, dav_tol):
    """The paper's convergence scheme for its carbon-dimer runs (section
    "Convergence scheme", Table 1: D 200 -> 2500, noise 0.03 then 0, E_conv
    1e-8, at most 47 sweeps) on the headline problem, stage by stage
    (sadmrg_solve_extrapolated), and the discarded-weight extrapolation
    (section "Extrapolation") through the noise-free stages."""
    from paper_1312_2415_amd import SaDMRG
    from paper_1312_2415_amd.binding import fit_discarded_weight
    from synth.integrals import make_integrals
    I = make_integrals(L, "D2h", seed)
    g = SaDMRG(L, 8, I.orb_irrep, device=0)
    try:
        g.set_integrals(I.h, I.eri)
        g.set_target(N, twoS, irrep)
        g.set_davidson(dav_tol, 32, 100)
        g.set_seed(seed)
        t = time.perf_counter()
        stages = []
        for k, ins in enumerate(TABLE1):
            n0 = len(g.trace())
            ts = time.perf_counter()
            e0, c1, pts = g.solve_extrapolated([ins])
            ts = time.perf_counter() - ts
            n_sw = (len(g.trace()) - n0) // (2 * (L - 1))
            stages.append({"D": ins[0], "noise": ins[3], "max_sweeps": ins[2], "sweeps": n_sw, "seconds": ts,
                           "w_disc": pts[0][1], "energy_last_sweep": pts[0][2]})
            print(f"scheme stage {k}: D={ins[0]} noise={ins[3]} {n_sw} sweeps {ts:.1f}s E={pts[0][2]:.10f} "
                  f"w={pts[0][1]:.3e}", file=sys.stderr, flush=True)
        t = time.perf_counter() - t
        e_min = g.energy()[0]
    finally:
        g.close()
    clean = [(st["w_disc"], st["energy_last_sweep"]) for st in stages if st["noise"] == 0.0]
    e0, c1 = fit_discarded_weight(clean)
    return {"workload": f"Table 1 convergence scheme on L={L} N={N} 2S={twoS} D2h irrep {irrep}, seeded synthetic "
                        f"integrals (seed {seed})",
            "seconds": t, "sweeps": sum(st["sweeps"] for st in stages), "energy_min": e_min,
            "extrapolated_energy": e0, "extrapolation_slope": c1, "stages": stages,
            "paper_context": "about 8 h per carbon-dimer geometry for this scheme on 16 Sandy Bridge cores "
                             "(cc-pVDZ integrals, not available here)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--L", type=int, default=28)
    ap.add_argument("--N", type=int, default=12)
    ap.add_argument("--twoS", type=int, default=0)
    ap.add_argument("--irrep", type=int, default=0)
    ap.add_argument("--D", type=int, default=2500)
    ap.add_argument("--copy-probe-mib", type=int, default=1024,
                    help="size of the reference streaming copy (HBM counter scale); 0 = skip")
    ap.add_argument("--gemm-probe", type=int, default=4096,
                    help="independent 64x256x64 products of the reference GEMM (counter scale); 0 = skip")
    ap.add_argument("--seed", type=int, default=1003)
    ap.add_argument("--dav-tol", type=float, default=1e-7)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-tol", type=float, default=1e-5)
    ap.add_argument("--mixed-steps", type=int, default=4, help="sweeps of each mixed-precision record (at most "
                                                               "--steps)")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-renorm32", action="store_true", help="skip the FP32-renormalisation mixed record")
    ap.add_argument("--no-rdm", action="store_true")
    ap.add_argument("--no-method-count", action="store_true")
    ap.add_argument("--batch-n", type=int, default=64, help="independent problems of the lockstep batch; 0 = skip")
    ap.add_argument("--batch-seed", type=int, default=4)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--only-batch", action="store_true", help="run only the lockstep batch record")
    ap.add_argument("--graph", type=int, default=4, help="replays per host check of the recorded Davidson "
                                                          "iterations in the batch record (0 = skip)")
    ap.add_argument("--roots", type=int, default=3, help="lockstep group size of the twelve-root record "
                                                         "(a divisor of 12; 0 = skip)")
    ap.add_argument("--roots-warmup", type=int, default=2)
    ap.add_argument("--refine", type=int, default=4, help="FP64 Davidson steps after the reduced-precision phase "
                                                          "(at most, with --refine-tol)")
    ap.add_argument("--only-roots", action="store_true", help="run only the roots record")
    ap.add_argument("--refine-tol", type=float, default=5e-7, help="FP64 residual norm that ends the refinement "
                                                                    "early (0 = always --refine steps)")
    ap.add_argument("--grad", type=int, default=4, help="integral orbits checked one by one by finite differences "
                                                        "in the energy-adjoint record at --grad-L orbitals (0 = skip)")
    ap.add_argument("--grad-dir", type=int, default=200, help="entries of the one multi-entry difference direction")
    ap.add_argument("--grad-L", type=int, default=36)
    ap.add_argument("--grad-warmup", type=int, default=3)
    ap.add_argument("--grad-tau", type=float, default=1e-5)
    ap.add_argument("--ckpt", type=int, default=6, help="block checkpoint interval of the operator-recomputation "
                                                        "leg of the grad record (0 = skip)")
    ap.add_argument("--only-grad", action="store_true", help="run only the energy-adjoint record")
    ap.add_argument("--scf-iter", type=int, default=2, help="DMRG-SCF iterations of the dmrgscf record (0 = skip)")
    ap.add_argument("--scf-D", type=int, default=1000)
    ap.add_argument("--scf-core", type=int, default=2)
    ap.add_argument("--only-dmrgscf", action="store_true")
    ap.add_argument("--only-scheme", action="store_true", help="run only the Table 1 convergence-scheme record")
    ap.add_argument("--gpc", default="", help="fixed sigma launch shape 'pass1,pass2' (workgroups per CU) "
                                               "instead of autotuning")
    ap.add_argument("--order", type=int, default=0, help="contraction order of the sigma products: 0 fewer flops, "
                                                          "1 fewer bytes streamed")
    ap.add_argument("--xcd", default="", help="XCD-grouped workgroup order of the sigma passes 'pass1,pass2' "
                                               "(0/1 each)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the method runs on a single MI355X here "
              "(sharding the sigma product over several GPUs is not run).",
              file=sys.stderr)
        sys.exit(2)

    if args.only_grad:
        print(json.dumps({"grad": grad_bench(args.grad_L, args.N, args.D, args.seed, args.grad_warmup,
                                             max(args.grad, 1), args.grad_tau, args.grad_dir, args.ckpt)}),
              flush=True)
        return
    if args.only_roots:
        print(json.dumps({"roots": roots_bench(args.roots, args.L, args.N, args.D, args.seed, args.roots_warmup,
                                               args.dav_tol, args.mixed_tol, args.refine, args.refine_tol)}),
              flush=True)
        return
    if args.only_batch:  # the lockstep batch record alone (for profiling it)
        print(json.dumps({"batch": batch_bench(max(args.batch_n, 1), args.batch_seed, 1, args.mixed_tol, args.graph)}),
              flush=True)
        return
    if args.only_dmrgscf:
        print(json.dumps({"dmrgscf": dmrgscf_bench(args.grad_L, args.N, args.scf_D, args.seed, args.scf_core,
                                                   max(args.scf_iter, 1), 2, args.dav_tol)}), flush=True)
        return
    if args.only_scheme:
        print(json.dumps({"scheme": scheme_bench(args.L, args.N, args.twoS, args.irrep, args.seed, args.dav_tol)}),
              flush=True)
        return

    from paper_1312_2415_amd import SaDMRG
    from synth.integrals import make_integrals

    L, N = args.L, args.N
    I = make_integrals(L, "D2h", args.seed)
    g = SaDMRG(L, 8, I.orb_irrep, device=0)
    g.set_integrals(I.h, I.eri)
    g.set_target(N, args.twoS, args.irrep)
    g.set_davidson(args.dav_tol, 32, 100)
    copy_gbps = None
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 8
        sec = g.copy_probe(n, 5)
        copy_gbps = 16.0 * n / sec / 1e9
        print(f"copy probe {args.copy_probe_mib} MiB: {1e3 * sec:.3f} ms/launch, {copy_gbps:.0f} GB/s", file=sys.stderr,
              flush=True)
    gemm_probe = None
    if args.gemm_probe > 0:
        sec, byt = g.gemm_probe(args.gemm_probe, 256, 5)
        gemm_probe = {"products": args.gemm_probe, "K": 256, "bytes_per_launch": byt, "ms_per_launch": 1e3 * sec,
                      "GBps": byt / sec / 1e9,
                      "kernel": "gemm_tile_kernel<double, 0>, the first dispatches of the run (5 launches)"}
        print(f"gemm probe {args.gemm_probe} products: {1e3 * sec:.3f} ms/launch, {byt / sec / 1e9:.0f} GB/s",
              file=sys.stderr, flush=True)
    xcd = None
    if args.xcd:
        xcd = [int(v) for v in args.xcd.split(",")]
        g.set_xcd_order(*xcd)
    g.set_contraction_order(args.order)
    g.init_mps(args.D)
    for w in range(args.warmup):
        t = time.time()
        e, _ = g.sweep(args.D)
        print(f"warmup sweep {w + 1}/{args.warmup} D={args.D} E={e:.10f} {time.time() - t:.1f}s", file=sys.stderr,
              flush=True)
    start = g.mps_export()  # the mixed sweeps restart from here
    # launch-shape autotuning on a middle step of the warmed-up MPS
    tune = None
    if args.gpc:
        g1, g2 = (int(v) for v in args.gpc.split(","))
        g.set_launch_shape(g1, g2)
        g.mps_import(start)
        tune = {"fixed_gpc_pass1_pass2": [g1, g2]}
    elif not args.no_autotune:
        g.advance(args.D, L // 2 - 1)
        g.prepare_step()
        chosen, table = g.autotune(5)
        g.mps_import(start)
        tune = {"step": L // 2 - 1, "chosen_gpc_pass1_pass2": list(chosen),
                "candidates_ms_per_sigma": {f"{a},{b}": ms for (a, b), ms in table}}
        print(f"autotune: pass-1/pass-2 workgroups per CU {chosen}", file=sys.stderr, flush=True)
    g.stats_reset()
    n_before = len(g.trace())
    t0 = time.perf_counter()
    energies = []
    # the FP64 state after as many sweeps as the mixed records run, for their
    # RDM comparison (its export is excluded from the timed window)
    nmix_ref = max(1, min(args.steps, args.mixed_steps))
    blob_nmix, t_export = None, 0.0
    for k in range(args.steps):
        ts = time.perf_counter()
        e, _ = g.sweep(args.D)
        energies.append(e)
        print(f"timed sweep {k + 1}/{args.steps} D={args.D} E={e:.10f} {time.perf_counter() - ts:.1f}s",
              file=sys.stderr, flush=True)
        if k + 1 == nmix_ref and not args.no_mixed and not args.no_rdm:
            tx = time.perf_counter()
            blob_nmix = g.mps_export()
            t_export += time.perf_counter() - tx
    t1 = time.perf_counter() - t_export
    from paper_1312_2415_amd.binding import device_memory
    mem_free, mem_total = device_memory(0)
    st = g.stats()
    trace64 = g.trace()
    per_sweep = 2 * (L - 1)
    sec_per_sweep = (t1 - t0) / args.steps
    sigma_tflops = st["flops_sigma"] / max(st["t_sigma"], 1e-12) / 1e12
    avg_sigma_ms = 1e3 * st["t_sigma"] / max(st["n_sigma"], 1)
    e_min, e_last, wd = g.energy()
    dom = max(("pass1", "pass2"), key=lambda k: st[k]["t"])
    ps = st[dom]
    nl = max(ps["launches"], 1)
    flops_per_launch = ps["flops"] / nl
    bytes_per_launch = ps["bytes"] / nl
    launch_ms = 1e3 * ps["t"] / nl
    achieved_tf = flops_per_launch / max(launch_ms, 1e-12) / 1e9
    achieved_gbs = bytes_per_launch / max(launch_ms, 1e-12) / 1e6
    ai = flops_per_launch / max(bytes_per_launch, 1.0)
    ridge = FP64_MFMA_PEAK / (HBM_PEAK / 1000.0)  # flop per byte where the two roofs meet
    if ai < ridge:
        roof = {"bound": "hbm", "achieved": achieved_gbs, "peak": HBM_PEAK, "unit": "GB/s",
                "frac": achieved_gbs / HBM_PEAK}
    else:
        roof = {"bound": "mfma", "achieved": achieved_tf, "peak": FP64_MFMA_PEAK, "unit": "TFLOP/s",
                "frac": achieved_tf / FP64_MFMA_PEAK}
    roof.update({"traffic": stored_traffic(dom), "kernel": PASS_KERNEL[dom], "flops_per_launch": flops_per_launch,
                 "algorithmic_bytes_per_launch": bytes_per_launch, "arithmetic_intensity": ai,
                 "ridge_flop_per_byte": ridge, "launch_ms_avg": launch_ms, "launches": ps["launches"],
                 "mfma_tflops": achieved_tf, "mfma_frac": achieved_tf / FP64_MFMA_PEAK})
    line = {
        "metric": METRIC,
        "value": sigma_tflops,
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * sec_per_sweep,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"spin-adapted two-site DMRG sweep, L={L} N={N} 2S={args.twoS} D2h irrep {args.irrep}, "
                               f"D_SU(2)={args.D}, seeded synthetic integrals (seed {args.seed})",
                   "L": L, "N": N, "twoS": args.twoS, "D": args.D, "point_group": "D2h",
                   "davidson_tol": args.dav_tol},
        "s_per_sweep": sec_per_sweep,
        "sigma_calls": st["n_sigma"],
        "sigma_ms_avg": avg_sigma_ms,
        "energy_min": e_min,
        "energy_last_sweep": energies[-1],
        "wdisc_max": wd,
        "sigma_passes": {k: {"ms_per_launch": 1e3 * st[k]["t"] / max(st[k]["launches"], 1),
                             "tflops": st[k]["flops"] / max(st[k]["t"], 1e-12) / 1e12,
                             "GBps_algorithmic": st[k]["bytes"] / max(st[k]["t"], 1e-12) / 1e9,
                             "arithmetic_intensity": st[k]["flops"] / max(st[k]["bytes"], 1.0),
                             "share_of_sigma_time": st[k]["t"] / max(st["t_sigma"], 1e-12)}
                         for k in ("pass1", "pass2")},
        "copy_probe_GBps": copy_gbps,
        "gemm_probe": gemm_probe,
        "autotune": tune,
        "xcd_order_pass1_pass2": xcd,
        "contraction_order": "fewer bytes streamed" if args.order == 1 else "fewer flops",
        "host_phase_seconds_per_sweep": {k: v / args.steps for k, v in st["phases"].items()},
        "davidson_sigma_seconds_per_sweep": st["t_sigma"] / args.steps,
        "max_enlarged_bytes": st["max_enlarged_bytes"],
        "device_memory_used_GiB_after_timed_sweeps": (mem_total - mem_free) / 2**30,
        "roofline": roof,
    }
    rdm64 = None
    if not args.no_rdm:  # spin-summed 1- and 2-RDM of the final FP64 MPS (energy adjoint)
        tr0 = time.perf_counter()
        ga, gb, g1, s2, e_rdm = g.calc2dm()
        t_rdm = time.perf_counter() - tr0
        rdm64 = (g1, ga)
        e_id = I.e_const + float(np.einsum("pq,pq", I.h, g1)) + 0.5 * float(np.einsum("ikjl,ijkl", I.eri, ga))
        line["rdm"] = {"seconds": t_rdm, "energy": e_rdm, "energy_identity_error": abs(e_id - e_rdm),
                       "trace_gamma": float(np.trace(g1)), "s2": s2,
                       "s2_error": abs(s2 - 0.25 * args.twoS * (args.twoS + 2))}
        print(f"rdm {t_rdm:.1f}s E={e_rdm:.10f} identity error {abs(e_id - e_rdm):.2e} <S^2> {s2:.2e}",
              file=sys.stderr, flush=True)
    if not args.no_method_count:
        # one more FP64 sweep with the method-work counter on (not timed): the
        # share of the performed sigma flops that multiply structurally
        # nonzero piece pairs of the enlarged operators
        g.set_method_counter(True)
        g.stats_reset()
        tm = time.perf_counter()
        g.sweep(args.D)
        tm = time.perf_counter() - tm
        mf, pf, _ = g.stats_method()
        g.set_method_counter(False)
        ratio = pf / max(mf, 1.0)
        line["method_work"] = {"performed_over_method_flops": ratio,
                               "sigma_method_tflops": sigma_tflops / ratio,
                               "counting_sweep_seconds": tm}
        roof["method_mfma_tflops"] = achieved_tf / ratio
        roof["method_mfma_frac"] = achieved_tf / ratio / FP64_MFMA_PEAK
        print(f"method work: performed / method flops {ratio:.3f}", file=sys.stderr, flush=True)
    if not args.no_mixed:
        # the first sweeps again from the same state with reduced-precision
        # sigma in Davidson (FP32, then BF16x3) and an FP64 refinement step
        nmix = nmix_ref
        rdm_nmix = None  # the FP64 RDMs after the same number of sweeps
        if blob_nmix is not None:
            g.mps_import(blob_nmix)
            r1, r2, _ = g.rdm()
            rdm_nmix = (r1, r2)
        ref_trace = trace64[n_before:n_before + nmix * per_sweep]
        for mode, key, desc, rprec in (
                (1, "mixed", "FP32 sigma (FP32 operators, FP32 accumulation) in Davidson", 0),
                (2, "mixed_bf16x3", "BF16x3 sigma (hi*hi + hi*lo + lo*hi of BF16 splits of the FP32 operators, "
                                    "FP32 accumulation) in Davidson", 0),
                (1, "mixed_fp32_renorm", "FP32 sigma in Davidson and FP32 renormalisation products (the new "
                                         "blocks stored in FP64 but carrying FP32 rounding)", 1)):
            if rprec and args.no_renorm32:
                continue
            g.set_renorm_precision(rprec)
            g.set_precision(mode, args.mixed_tol)
            g.set_refinement(args.refine)
            g.set_refinement_tol(args.refine_tol)
            g.mps_import(start)
            g.stats_reset()
            n_done = len(g.trace())
            tm0 = time.perf_counter()
            emix = []
            for k in range(nmix):
                ts = time.perf_counter()
                e, _ = g.sweep(args.D)
                emix.append(e)
                print(f"{key} sweep {k + 1}/{nmix} D={args.D} E={e:.10f} {time.perf_counter() - ts:.1f}s",
                      file=sys.stderr, flush=True)
            tm1 = time.perf_counter()
            sm = g.stats()
            tracem = g.trace()[n_done:n_done + len(ref_trace)]
            d_micro = float(np.abs(np.array(tracem) - np.array(ref_trace)).max()) \
                if len(tracem) == len(ref_trace) and len(ref_trace) else None
            sec_mixed = (tm1 - tm0) / nmix
            peak = FP32_MFMA_PEAK if mode == 1 else BF16_MFMA_PEAK / 3
            tf = sm["fp32"]["flops"] / max(sm["fp32"]["t"], 1e-12) / 1e12
            rec = {
                "precision": desc + f"; FP64 Davidson algebra and SVD{'' if rprec else ', FP64 renormalisation'}; "
                                    f"up to {args.refine} FP64 Davidson step(s) (until the FP64 residual is "
                                    f"<= {args.refine_tol:g}) refine each micro-iteration's vector and give its energy",
                "mixed_tol": args.mixed_tol,
                "fp64_refinement_steps": args.refine,
                "fp64_refinement_residual_target": args.refine_tol,
                "renormalisation": "FP32" if rprec else "FP64",
                "sweeps": nmix,
                "s_per_sweep": sec_mixed,
                "speedup_s_per_sweep": sec_per_sweep / sec_mixed,
                "sigma_reduced_tflops": tf,
                "sigma_reduced_roofline_frac": tf / peak,
                "sigma_reduced_peak_tflops": peak,
                "sigma_reduced_calls": sm["fp32"]["calls"],
                "sigma_fp64_calls": sm["n_sigma"],
                "sigma_seconds_per_sweep": (sm["fp32"]["t"] + sm["t_sigma"]) / nmix,
                "sigma_seconds_per_sweep_fp64_path": st["t_sigma"] / args.steps,
                "energy_last_sweep": emix[-1],
                "abs_dE_last_sweep_vs_fp64": abs(emix[-1] - energies[nmix - 1]),
                "max_abs_dE_per_micro_iteration_vs_fp64": d_micro,
            }
            if rdm_nmix is not None:
                m1, m2, _ = g.rdm()
                rec["rdm_max_abs_error_vs_fp64"] = {"gamma": float(np.abs(m1 - rdm_nmix[0]).max()),
                                                    "Gamma": float(np.abs(m2 - rdm_nmix[1]).max())}
            line[key] = rec
        g.set_renorm_precision(0)
    if args.graph > 0:
        # the first timed FP64 sweeps again from the same state with the
        # Davidson iterations replayed from a recorded HIP graph
        nrec = max(1, min(args.steps, 2))
        g.set_precision(0, args.mixed_tol)
        g.set_davidson_graph(args.graph)
        g.mps_import(start)
        g.stats_reset()
        n_done = len(g.trace())
        tg0 = time.perf_counter()
        for k in range(nrec):
            ts = time.perf_counter()
            e, _ = g.sweep(args.D)
            print(f"recorded-Davidson sweep {k + 1}/{nrec} D={args.D} E={e:.10f} {time.perf_counter() - ts:.1f}s",
                  file=sys.stderr, flush=True)
        tg1 = time.perf_counter()
        sgr = g.stats_graph()
        trg = np.array(g.trace()[n_done:n_done + nrec * per_sweep])
        ref = np.array(trace64[n_before:n_before + nrec * per_sweep])
        line["recorded_davidson"] = {
            "replays_per_host_check": args.graph, "sweeps": nrec,
            "s_per_sweep": (tg1 - tg0) / nrec, "speedup_vs_host_driven": sec_per_sweep / ((tg1 - tg0) / nrec),
            "replayed_segment_seconds_per_sweep": sgr["seconds"] / nrec,
            "recording_host_seconds_per_sweep": sgr["record_seconds"] / nrec,
            "sigma_products_in_replays": sgr["sigma_calls"], "recordings": sgr["records"],
            "trace_identical_to_host_driven": bool(len(trg) == len(ref) and np.array_equal(trg, ref)),
        }
        g.set_davidson_graph(0)
    g.close()
    if args.batch_n > 0:
        line["batch"] = batch_bench(args.batch_n, args.batch_seed, 1, args.mixed_tol, args.graph)
    # the extra records run last; after a failed record no further GPU work
    # that fills the device is started
    failed = False
    for key, run in (("grad", lambda: grad_bench(args.grad_L, N, args.D, args.seed, args.grad_warmup, args.grad,
                                                 args.grad_tau, args.grad_dir, args.ckpt) if args.grad > 0 else None),
                     ("dmrgscf", lambda: dmrgscf_bench(args.grad_L, N, args.scf_D, args.seed, args.scf_core,
                                                       args.scf_iter, 2, args.dav_tol) if args.scf_iter > 0 else None),
                     ("roots", lambda: roots_bench(args.roots, L, N, args.D, args.seed, args.roots_warmup,
                                                   args.dav_tol, args.mixed_tol, args.refine, args.refine_tol)
                      if args.roots > 0 else None)):
        if failed:
            break
        try:
            rec = run()
            if rec is not None:
                line[key] = rec
        except Exception as ex:  # the headline record stands on its own
            line[key] = {"error": f"{type(ex).__name__}: {ex}"}
            failed = True
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, L, N, args.twoS, args.irrep, args.seed, args.D,
                                            L // 2 - 1)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
