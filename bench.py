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


def cpu_baseline(seconds: float, L: int, N: int, twoS: int, irrep: int, seed: int, D: int):
    """The oracle's sigma rate on a bounded sample of the same workload.

    Sample: the oracle DMRG on the same integrals and target with bond
    dimension D (boundary blocks built), then micro-iterations of the first
    left-to-right pass until `seconds` of sigma time; flops are counted with the
    GPU path's definition (dense enlarged-block triple products, each in the
    cheaper of its two contraction orders).
    """
    import numpy as np

    from oracle import sadmrg as sd
    from synth.integrals import make_integrals

    I = make_integrals(L, "D2h", seed)
    P = sd.Problem(I.h, I.eri, N, twoS, irrep, I.orb_irrep)
    dm = sd.DMRG(P, D, seed=3)
    dm.build_boundaries()
    acc = {"t": 0.0, "f": 0.0, "n": 0}
    orig_apply = sd.Heff.apply

    def flops_of(H):
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
                # the cheaper contraction order, as the GPU path chooses it
                f += mult * min(2.0 * R * K2 * (K1 + C), 2.0 * K1 * C * (K2 + R))
        return f

    def timed_apply(self, psi):
        if not hasattr(self, "dx"):
            self.dx = {m: v.shape[0] for m, v in psi.items()}
            self.dy = {m: v.shape[1] for m, v in psi.items()}
            self._f = flops_of(self)
        t = time.perf_counter()
        out = orig_apply(self, psi)
        acc["t"] += time.perf_counter() - t
        acc["f"] += self._f
        acc["n"] += 1
        return out

    sd.Heff.apply = timed_apply
    steps = 0
    try:
        for i in range(0, L - 2):
            dm.micro(i, D, "right")
            steps += 1
            if acc["t"] >= seconds:
                break
    finally:
        sd.Heff.apply = orig_apply
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        cores = 1
    rate = acc["f"] / max(acc["t"], 1e-12) / 1e12
    return {"value": rate, "unit": "TFLOP/s", "cores": int(cores), "kind": "oracle",
            "sample": f"oracle sigma on L={L} N={N} 2S={twoS} D2h, D={D}: {acc['n']} sigma calls over the first "
                      f"{steps} micro-iterations of a left-to-right pass ({acc['t']:.1f} s of sigma time); "
                      f"flops counted as for the GPU path", "sigma_calls": acc["n"],
            "sigma_seconds": acc["t"]}


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


def batch_bench(n, seed, prec, mixed_tol):
    """One lockstep sweep of n problems (sadmrg_batch_sweep) against the same
    problems swept one after another from the same states."""
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
        "L": [sp["L"] for sp in specs], "D": Ds,
    }


ROOT_TARGETS = [(2 * s, ir) for s in (0, 1, 2) for ir in (0, 1, 2, 3)]  # (2S, irrep) of the twelve roots


def roots_bench(k, L, N, D, seed, warm, dav_tol, mixed_tol, refine=1):
    """Roots 0, 12/k, 2*12/k, ... of the twelve (one GPU's share when they are
    dealt round-robin over 12/k GPUs) swept in lockstep (sadmrg_batch_sweep):
    `warm` FP64 lockstep sweeps from random MPS, then one timed FP64 lockstep
    sweep, the same sweep of each root on its own, and one timed mixed
    lockstep sweep (FP32 sigma + FP64 refinement) from the same states."""
    from paper_1312_2415_amd import SaDMRG
    from paper_1312_2415_amd.binding import batch_sweep, device_memory
    from synth.integrals import make_integrals
    if k < 1 or 12 % k:
        raise ValueError("roots: k must divide 12")
    targets = ROOT_TARGETS[::12 // k]
    I = make_integrals(L, "D2h", seed)
    gs = []
    try:
        for j, (twoS, irrep) in enumerate(targets):
            g = SaDMRG(L, 8, I.orb_irrep, device=0)
            gs.append(g)
            g.set_integrals(I.h, I.eri)
            g.set_target(N, twoS, irrep)
            g.set_seed(seed + 17 * j)
            g.set_davidson(dav_tol, 32, 100)
            g.init_mps(D)
        for w in range(warm):
            t = time.perf_counter()
            batch_sweep(gs, D)
            print(f"roots: warm-up lockstep sweep {w + 1}/{warm} {time.perf_counter() - t:.1f}s", file=sys.stderr,
                  flush=True)
        blobs = [g.mps_export() for g in gs]
        n0 = [len(g.trace()) for g in gs]
        t = time.perf_counter()
        e64, st64, _ = batch_sweep(gs, D)
        t64 = time.perf_counter() - t
        free, total = device_memory(0)
        tr64 = [np.array(g.trace()[n:]) for g, n in zip(gs, n0)]
        print(f"roots: FP64 lockstep sweep {t64:.2f}s", file=sys.stderr, flush=True)
        r64 = [g.rdm() for g in gs]
        t = time.perf_counter()
        for g, b in zip(gs, blobs):
            g.mps_import(b)
            g.sweep(D)
        tsep = time.perf_counter() - t
        print(f"roots: separate FP64 sweeps {tsep:.2f}s", file=sys.stderr, flush=True)
        n1 = []
        for g, b in zip(gs, blobs):
            g.set_precision(1, mixed_tol)
            g.set_refinement(refine)
            g.mps_import(b)
            n1.append(len(g.trace()))
        t = time.perf_counter()
        e32, st32, _ = batch_sweep(gs, D)
        t32 = time.perf_counter() - t
        tr32 = [np.array(g.trace()[n:]) for g, n in zip(gs, n1)]
        print(f"roots: mixed lockstep sweep {t32:.2f}s", file=sys.stderr, flush=True)
        r32 = [g.rdm() for g in gs]
        per = []
        for j, (twoS, irrep) in enumerate(targets):
            same = len(tr32[j]) == len(tr64[j]) and len(tr64[j]) > 0
            per.append({"twoS": twoS, "irrep": irrep, "energy_fp64": e64[j], "energy_mixed": e32[j],
                        "abs_dE": abs(e32[j] - e64[j]),
                        "max_abs_dE_per_micro_iteration": float(np.abs(tr32[j] - tr64[j]).max()) if same else None,
                        "rdm_max_abs_error": {"gamma": float(np.abs(r32[j][0] - r64[j][0]).max()),
                                              "Gamma": float(np.abs(r32[j][1] - r64[j][1]).max())}})
        f64 = st64["flops_sigma"] / max(st64["t_sigma"], 1e-12) / 1e12
        f32 = st32["flops_sigma32"] / max(st32["t_sigma32"], 1e-12) / 1e12
        return {
            "workload": f"roots of L={L} N={N} D2h D_SU(2)={D} (seed {seed}): (2S, irrep) in "
                        f"{[list(t) for t in targets]}, the share of one GPU when the twelve roots "
                        f"(S in {{0,1,2}} x irreps 0..3) are dealt round-robin to {12 // k} GPUs",
            "roots": k, "warmup_lockstep_sweeps": warm, "fp64_refinement_steps": refine,
            "s_per_lockstep_sweep_fp64": t64,
            "s_per_separate_sweeps_fp64": tsep,
            "s_per_lockstep_sweep_mixed": t32,
            "speedup_mixed_lockstep_vs_fp64_lockstep": t64 / t32,
            "speedup_mixed_lockstep_vs_fp64_separate": tsep / t32,
            "sigma_tflops_fp64_lockstep": f64,
            "sigma_roofline_frac_fp64": f64 / FP64_MFMA_PEAK,
            "sigma_tflops_fp32_mixed": f32,
            "sigma_roofline_frac_fp32": f32 / FP32_MFMA_PEAK,
            "max_abs_dE": max(r["abs_dE"] for r in per),
            "max_rdm_abs_error": max(max(r["rdm_max_abs_error"].values()) for r in per),
            "device_memory_used_GiB": (total - free) / 2**30,
            "per_root": per,
        }
    finally:
        for g in gs:
            g.close()


def grad_bench(L, N, D, seed, warm, n_orbits, tau):
    """Energy adjoint at the differentiation configuration (L orbitals, N
    electrons, singlet Ag, D2h): the spin-summed 1- and 2-RDM of the MPS after
    `warm` sweeps at D, as dE/dh and dE/d(ij|kl), against central differences
    of E = <psi|H|psi> for that same frozen MPS along symmetry-allowed integral
    orbits (every evaluation rebuilds all renormalised operators from the MPS
    with the shifted integrals).  At fixed psi, E is linear in the integrals,
    so the difference quotient is exact up to rounding."""
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
        t_fd = time.perf_counter() - t_fd
        return {
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
    ap.add_argument("--seed", type=int, default=1003)
    ap.add_argument("--dav-tol", type=float, default=1e-7)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-D", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--mixed-tol", type=float, default=1e-5)
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-rdm", action="store_true")
    ap.add_argument("--batch-n", type=int, default=64, help="independent problems of the lockstep batch; 0 = skip")
    ap.add_argument("--batch-seed", type=int, default=4)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--only-batch", action="store_true", help="run only the lockstep batch record")
    ap.add_argument("--roots", type=int, default=3, help="roots of the headline problem swept in lockstep "
                                                         "(a divisor of 12; 0 = skip)")
    ap.add_argument("--roots-warmup", type=int, default=2)
    ap.add_argument("--refine", type=int, default=1, help="FP64 Davidson steps after the reduced-precision phase")
    ap.add_argument("--only-roots", action="store_true", help="run only the roots record")
    ap.add_argument("--grad", type=int, default=4, help="integral orbits checked by finite differences in the "
                                                        "energy-adjoint record at --grad-L orbitals (0 = skip)")
    ap.add_argument("--grad-L", type=int, default=36)
    ap.add_argument("--grad-warmup", type=int, default=3)
    ap.add_argument("--grad-tau", type=float, default=1e-5)
    ap.add_argument("--only-grad", action="store_true", help="run only the energy-adjoint record")
    ap.add_argument("--gpc", default="", help="fixed sigma launch shape 'pass1,pass2' (workgroups per CU) "
                                               "instead of autotuning")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the method runs on a single MI355X here "
              "(sharding the sigma product over several GPUs is not run).",
              file=sys.stderr)
        sys.exit(2)

    if args.only_grad:
        print(json.dumps({"grad": grad_bench(args.grad_L, args.N, args.D, args.seed, args.grad_warmup,
                                             max(args.grad, 1), args.grad_tau)}), flush=True)
        return
    if args.only_roots:
        print(json.dumps({"roots": roots_bench(args.roots, args.L, args.N, args.D, args.seed, args.roots_warmup,
                                               args.dav_tol, args.mixed_tol, args.refine)}), flush=True)
        return
    if args.only_batch:  # the lockstep batch record alone (for profiling it)
        print(json.dumps({"batch": batch_bench(max(args.batch_n, 1), args.batch_seed, 1, args.mixed_tol)}),
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
    import numpy as np
    g.stats_reset()
    t0 = time.perf_counter()
    energies = []
    for k in range(args.steps):
        ts = time.perf_counter()
        e, _ = g.sweep(args.D)
        energies.append(e)
        print(f"timed sweep {k + 1}/{args.steps} D={args.D} E={e:.10f} {time.perf_counter() - ts:.1f}s",
              file=sys.stderr, flush=True)
    t1 = time.perf_counter()
    from paper_1312_2415_amd.binding import device_memory
    mem_free, mem_total = device_memory(0)
    st = g.stats()
    trace64 = g.trace()
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
    achieved = flops_per_launch / max(launch_ms, 1e-12) / 1e9
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
                             "share_of_sigma_time": st[k]["t"] / max(st["t_sigma"], 1e-12)}
                         for k in ("pass1", "pass2")},
        "copy_probe_GBps": copy_gbps,
        "autotune": tune,
        "host_phase_seconds_per_sweep": {k: v / args.steps for k, v in st["phases"].items()},
        "davidson_sigma_seconds_per_sweep": st["t_sigma"] / args.steps,
        "max_enlarged_bytes": st["max_enlarged_bytes"],
        "device_memory_used_GiB_after_timed_sweeps": (mem_total - mem_free) / 2**30,
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": FP64_MFMA_PEAK, "unit": "TFLOP/s",
                     "frac": achieved / FP64_MFMA_PEAK, "traffic": stored_traffic(dom),
                     "kernel": PASS_KERNEL[dom], "flops_per_launch": flops_per_launch,
                     "algorithmic_bytes_per_launch": bytes_per_launch, "launch_ms_avg": launch_ms,
                     "launches": ps["launches"]},
    }
    rdm64 = None
    if not args.no_rdm:  # spin-summed 1- and 2-RDM of the final FP64 MPS (energy adjoint)
        tr0 = time.perf_counter()
        g1, g2, e_rdm = g.rdm()
        t_rdm = time.perf_counter() - tr0
        rdm64 = (g1, g2)
        e_id = I.e_const + float(np.einsum("pq,pq", I.h, g1)) + 0.5 * float(np.einsum("ikjl,ijkl", I.eri, g2))
        line["rdm"] = {"seconds": t_rdm, "energy": e_rdm, "energy_identity_error": abs(e_id - e_rdm),
                       "trace_gamma": float(np.trace(g1))}
        print(f"rdm {t_rdm:.1f}s E={e_rdm:.10f} identity error {abs(e_id - e_rdm):.2e}", file=sys.stderr, flush=True)
    if not args.no_mixed:
        # the same timed sweeps from the same state with reduced-precision
        # sigma in Davidson (FP32, then BF16x3) and an FP64 refinement step
        n_done = len(trace64)
        for mode, key, desc in (
                (1, "mixed", "FP32 sigma (FP32 operators, FP32 accumulation) in Davidson"),
                (2, "mixed_bf16x3", "BF16x3 sigma (hi*hi + hi*lo + lo*hi of BF16 splits of the FP32 operators, "
                                    "FP32 accumulation) in Davidson")):
            g.set_precision(mode, args.mixed_tol)
            g.set_refinement(args.refine)
            g.mps_import(start)
            g.stats_reset()
            tm0 = time.perf_counter()
            emix = []
            for k in range(args.steps):
                ts = time.perf_counter()
                e, _ = g.sweep(args.D)
                emix.append(e)
                print(f"{key} sweep {k + 1}/{args.steps} D={args.D} E={e:.10f} {time.perf_counter() - ts:.1f}s",
                      file=sys.stderr, flush=True)
            tm1 = time.perf_counter()
            sm = g.stats()
            tracem = g.trace()
            nt = len(tracem) - n_done  # micro-iterations of these sweeps
            d_micro = float(max(abs(a - b) for a, b in zip(trace64[len(trace64) - nt:], tracem[n_done:]))) \
                if nt > 0 else None
            n_done = len(tracem)
            sec_mixed = (tm1 - tm0) / args.steps
            peak = FP32_MFMA_PEAK if mode == 1 else BF16_MFMA_PEAK / 3
            tf = sm["fp32"]["flops"] / max(sm["fp32"]["t"], 1e-12) / 1e12
            rec = {
                "precision": desc + f"; FP64 Davidson algebra, SVD, renormalisation; {args.refine} FP64 Davidson "
                                    f"step(s) ({args.refine + 1} FP64 sigma) refine each micro-iteration's vector "
                                    "and give its energy",
                "mixed_tol": args.mixed_tol,
                "fp64_refinement_steps": args.refine,
                "s_per_sweep": sec_mixed,
                "speedup_s_per_sweep": sec_per_sweep / sec_mixed,
                "sigma_reduced_tflops": tf,
                "sigma_reduced_roofline_frac": tf / peak,
                "sigma_reduced_peak_tflops": peak,
                "sigma_reduced_calls": sm["fp32"]["calls"],
                "sigma_fp64_calls": sm["n_sigma"],
                "sigma_seconds_per_sweep": (sm["fp32"]["t"] + sm["t_sigma"]) / args.steps,
                "sigma_seconds_per_sweep_fp64_path": st["t_sigma"] / args.steps,
                "energy_last_sweep": emix[-1],
                "abs_dE_last_sweep_vs_fp64": abs(emix[-1] - energies[-1]),
                "max_abs_dE_per_micro_iteration_vs_fp64": d_micro,
            }
            if rdm64 is not None:
                m1, m2, _ = g.rdm()
                rec["rdm_max_abs_error_vs_fp64"] = {"gamma": float(np.abs(m1 - rdm64[0]).max()),
                                                    "Gamma": float(np.abs(m2 - rdm64[1]).max())}
            line[key] = rec
    g.close()
    if args.batch_n > 0:
        line["batch"] = batch_bench(args.batch_n, args.batch_seed, 1, args.mixed_tol)
    # the extra records run last, the one that fills device memory most at the
    # end; after a failed record no further GPU work is started
    if args.grad > 0:
        try:
            line["grad"] = grad_bench(args.grad_L, N, args.D, args.seed, args.grad_warmup, args.grad, args.grad_tau)
        except Exception as ex:  # the headline record stands on its own
            line["grad"] = {"error": f"{type(ex).__name__}: {ex}"}
    if args.roots > 0 and "error" not in line.get("grad", {}):
        try:
            line["roots"] = roots_bench(args.roots, L, N, args.D, args.seed, args.roots_warmup, args.dav_tol,
                                        args.mixed_tol, args.refine)
        except Exception as ex:
            line["roots"] = {"error": f"{type(ex).__name__}: {ex}"}
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds, L, N, args.twoS, args.irrep, args.seed, args.cpu_D)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
