"""ctypes binding of libsadmrg (argument marshalling only).

Every numerical step runs inside the HIP library; this module converts numpy
arrays / torch tensors to pointers and status codes to exceptions.  The
library is required: importing works without it, but constructing a solver
raises if ``libsadmrg.so`` has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None
_LIB_PATH = None

_ERR = {-1: "EINVAL", -2: "ESYMM", -3: "EINTEG", -4: "ENOMEM", -5: "EDEVICE"}


def library_path() -> str:
    return os.path.join(_HERE, "libsadmrg.so")


def load_library(path: str | None = None):
    """Load (once) and return the ctypes handle of libsadmrg."""
    global _LIB, _LIB_PATH
    path = os.path.abspath(path or library_path())
    if _LIB is not None and _LIB_PATH == path:
        return _LIB
    if not os.path.exists(path):
        raise RuntimeError(f"libsadmrg not built: {path} is missing (build it with python -m paper_1312_2415_amd.build)")
    # torch's wheel ships its own HIP runtime under the same soname as the
    # system one the library links; whichever is loaded first serves the whole
    # process.  Loading torch first gives the library the runtime that owns
    # torch's device tensors and streams (and keeps torch usable afterwards).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    c_int, c_dbl, c_vp, c_sz = ctypes.c_int, ctypes.c_double, ctypes.c_void_p, ctypes.c_size_t
    P = ctypes.POINTER
    sig = {
        "sadmrg_version": (ctypes.c_char_p, []),
        "sadmrg_create": (c_int, [P(c_vp), c_int, c_int, P(c_int), c_int]),
        "sadmrg_destroy": (None, [c_vp]),
        "sadmrg_set_stream": (c_int, [c_vp, c_vp]),
        "sadmrg_set_allocator": (c_int, [c_vp, c_vp, c_vp, c_vp]),
        "sadmrg_set_integrals": (c_int, [c_vp, c_dbl, P(c_dbl), P(c_dbl), c_dbl]),
        "sadmrg_set_target": (c_int, [c_vp, c_int, c_int, c_int]),
        "sadmrg_set_davidson": (c_int, [c_vp, c_dbl, c_int, c_int]),
        "sadmrg_set_seed": (c_int, [c_vp, ctypes.c_uint64]),
        "sadmrg_init_mps": (c_int, [c_vp, c_int]),
        "sadmrg_sweep": (c_int, [c_vp, c_int, P(c_dbl)]),
        "sadmrg_batch_sweep": (c_int, [P(c_vp), c_int, P(c_int), P(c_dbl), P(c_dbl)]),
        "sadmrg_solve": (c_int, [c_vp, c_int, P(c_int), P(c_dbl), P(c_int), P(c_dbl), P(c_dbl)]),
        "sadmrg_get_energy": (c_int, [c_vp, P(c_dbl), P(c_dbl), P(c_dbl)]),
        "sadmrg_set_contraction_order": (c_int, [c_vp, c_int]),
        "sadmrg_set_xcd_order": (c_int, [c_vp, c_int, c_int]),
        "sadmrg_debug_gemm_probe": (c_int, [c_vp, c_int, c_int, c_int, P(c_dbl), P(c_dbl)]),
        "sadmrg_set_method_counter": (c_int, [c_vp, c_int]),
        "sadmrg_stats_method": (c_int, [c_vp, P(c_dbl), P(c_dbl), P(c_dbl)]),
        "sadmrg_push_excitation": (c_int, [c_vp, c_dbl]),
        "sadmrg_clear_excitations": (c_int, [c_vp]),
        "sadmrg_rotate_integrals": (c_int, [c_int, P(c_dbl), P(c_dbl), P(c_dbl), P(c_dbl), P(c_dbl)]),
        "sadmrg_rotation": (c_int, [c_int, P(c_dbl), P(c_dbl)]),
        "sadmrg_orbital_derivatives": (c_int, [c_int, P(c_dbl), P(c_dbl), P(c_dbl), P(c_dbl), c_int, P(c_int),
                                               P(c_dbl), P(c_dbl), P(c_dbl)]),
        "sadmrg_dmrgscf": (c_int, [c_vp, c_int, P(c_int), P(c_int), c_dbl, P(c_dbl), P(c_dbl), c_int, P(c_int),
                                   P(c_dbl), P(c_int), P(c_dbl), c_dbl, c_int, c_dbl, P(c_dbl), P(c_dbl), P(c_int),
                                   P(c_dbl)]),
        "sadmrg_extrapolate": (c_int, [c_int, P(c_dbl), P(c_dbl), P(c_dbl), P(c_dbl)]),
        "sadmrg_solve_extrapolated": (c_int, [c_vp, c_int, P(c_int), P(c_dbl), P(c_int), P(c_dbl), P(c_dbl),
                                              P(c_dbl), P(c_dbl)]),
        "sadmrg_get_trace": (c_int, [c_vp, P(c_dbl), P(c_int)]),
        "sadmrg_mps_import": (c_int, [c_vp, c_vp, c_sz]),
        "sadmrg_mps_export": (c_int, [c_vp, c_vp, P(c_sz)]),
        "sadmrg_prepare_step": (c_int, [c_vp]),
        "sadmrg_advance": (c_int, [c_vp, c_int, c_int, P(c_dbl)]),
        "sadmrg_debug_task_shapes": (c_int, [c_vp, P(c_int), P(ctypes.c_int64)]),
        "sadmrg_psi_layout": (c_int, [c_vp, P(c_int), P(ctypes.c_int64), P(ctypes.c_int64)]),
        "sadmrg_sigma": (c_int, [c_vp, c_vp, c_vp, c_int]),
        "sadmrg_heff_diagonal": (c_int, [c_vp, c_vp, c_int]),
        "sadmrg_debug_guess": (c_int, [c_vp, c_vp, c_int]),
        "sadmrg_sigma_noalloc": (c_int, [c_vp, c_vp, c_vp]),
        "sadmrg_debug_plan_stats": (c_int, [c_vp, P(ctypes.c_int64)]),
        "sadmrg_sigma_counters": (c_int, [c_vp, P(c_dbl), P(c_dbl), P(ctypes.c_int64)]),
        "sadmrg_stats": (c_int, [c_vp, P(c_dbl), P(ctypes.c_int64), P(c_dbl), P(c_dbl), P(c_dbl)]),
        "sadmrg_stats_reset": (c_int, [c_vp]),
        "sadmrg_stats_phases": (c_int, [c_vp, P(c_dbl)]),
        "sadmrg_set_enlarge_cache": (c_int, [c_vp, c_int]),
        "sadmrg_device_memory": (c_int, [c_int, P(c_sz), P(c_sz)]),
        "sadmrg_autotune": (c_int, [c_vp, c_int, P(c_int), P(c_int), P(c_dbl)]),
        "sadmrg_set_launch_shape": (c_int, [c_vp, c_int, c_int]),
        "sadmrg_stats_bytes": (c_int, [c_vp, P(c_dbl), P(c_dbl)]),
        "sadmrg_stats_passes": (c_int, [c_vp, P(c_dbl), P(c_dbl)]),
        "sadmrg_stats_mixed": (c_int, [c_vp, P(c_dbl), P(ctypes.c_int64), P(c_dbl)]),
        "sadmrg_set_refinement": (c_int, [c_vp, c_int]),
        "sadmrg_set_block_checkpoints": (c_int, [c_vp, c_int]),
        "sadmrg_stats_blocks": (c_int, [c_vp, P(ctypes.c_int64), P(c_dbl), P(c_dbl), P(c_int)]),
        "sadmrg_set_davidson_graph": (c_int, [c_vp, c_int]),
        "sadmrg_stats_graph": (c_int, [c_vp, P(c_dbl), P(c_dbl), P(c_dbl), P(ctypes.c_int64), P(ctypes.c_int64),
                                       P(ctypes.c_int64)]),
        "sadmrg_set_renorm_precision": (c_int, [c_vp, c_int]),
        "sadmrg_set_refinement_tol": (c_int, [c_vp, c_dbl]),
        "sadmrg_set_precision": (c_int, [c_vp, c_int, c_dbl]),
        "sadmrg_rdm": (c_int, [c_vp, P(c_dbl), P(c_dbl), P(c_dbl)]),
        "sadmrg_get_s2": (c_int, [c_vp, P(c_dbl)]),
        "sadmrg_calc2dm": (c_int, [c_vp, P(c_dbl), P(c_dbl), c_int, P(c_dbl), P(c_dbl), P(c_dbl)]),
        "sadmrg_debug_copy_probe": (c_int, [c_vp, ctypes.c_int64, c_int, P(c_dbl)]),
        "sadmrg_last_error": (ctypes.c_char_p, [c_vp]),
        "sadmrg_debug_coupling": (c_int, [c_int, P(c_int), P(c_dbl)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _LIB, _LIB_PATH = lib, path
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class SadmrgError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_ERR.get(code, code)}: {msg}")
        self.code = code


class SaDMRG:
    """One solver context (one target sector) on one HIP device."""

    def __init__(self, L: int, group_order: int, orb_irrep, device: int = 0, lib_path: str | None = None):
        self.lib = load_library(lib_path)
        irr = np.ascontiguousarray(orb_irrep, dtype=np.int32)
        self.L = int(L)
        h = ctypes.c_void_p()
        rc = self.lib.sadmrg_create(ctypes.byref(h), int(L), int(group_order),
                                    irr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), int(device))
        if rc != 0:
            raise SadmrgError(rc, "sadmrg_create failed")
        self.h = h

    def close(self):
        if getattr(self, "h", None):
            self.lib.sadmrg_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc):
        if rc < 0:
            raise SadmrgError(rc, self.lib.sadmrg_last_error(self.h).decode())
        return rc

    # ---- problem definition
    ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p)
    FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p)

    def set_allocator(self, alloc, free):
        """sadmrg_set_allocator with Python callables alloc(bytes, device) -> int
        pointer (0 on failure) and free(ptr, bytes, device); None, None restores
        hipMalloc.  The callables are kept alive with the solver."""
        if alloc is None and free is None:
            self._hooks = None
            self._chk(self.lib.sadmrg_set_allocator(self.h, None, None, None))
            return
        a = self.ALLOC_FN(lambda n, dev, user: int(alloc(int(n), int(dev))) or None)
        f = self.FREE_FN(lambda p, n, dev, user: free(int(p), int(n), int(dev)))
        self._chk(self.lib.sadmrg_set_allocator(self.h, ctypes.cast(a, ctypes.c_void_p),
                                                ctypes.cast(f, ctypes.c_void_p), None))
        self._hooks = (a, f)

    def use_torch_allocator(self):
        """Route the context's device memory through torch's caching allocator
        (torch.cuda.caching_allocator_alloc / _delete on the current stream)."""
        import torch

        def alloc(n, dev):
            try:
                return torch.cuda.caching_allocator_alloc(n, device=dev)
            except RuntimeError:
                return 0

        self.set_allocator(alloc, lambda p, n, dev: torch.cuda.caching_allocator_delete(p))

    def set_stream(self, stream_handle: int):
        self._chk(self.lib.sadmrg_set_stream(self.h, ctypes.c_void_p(int(stream_handle))))

    def set_integrals(self, h, eri, e_const=0.0, sym_tol=1e-10):
        h = np.ascontiguousarray(h, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        if h.shape != (self.L, self.L) or eri.shape != (self.L,) * 4:
            raise ValueError("integral shapes do not match L")
        self._chk(self.lib.sadmrg_set_integrals(self.h, float(e_const), _dptr(h), _dptr(eri), float(sym_tol)))

    def set_target(self, N, twoS, irrep=0):
        self._chk(self.lib.sadmrg_set_target(self.h, int(N), int(twoS), int(irrep)))

    def set_davidson(self, tol=1e-9, max_sub=32, max_iter=200):
        self._chk(self.lib.sadmrg_set_davidson(self.h, float(tol), int(max_sub), int(max_iter)))

    def set_seed(self, seed):
        self._chk(self.lib.sadmrg_set_seed(self.h, ctypes.c_uint64(int(seed))))

    # ---- sweeping
    def init_mps(self, D):
        self._chk(self.lib.sadmrg_init_mps(self.h, int(D)))

    def sweep(self, D):
        e = ctypes.c_double()
        rc = self._chk(self.lib.sadmrg_sweep(self.h, int(D), ctypes.byref(e)))
        return e.value, rc

    def solve(self, schedule):
        """schedule: list of (D, e_conv, max_sweeps[, noise])."""
        n = len(schedule)
        D = (ctypes.c_int * n)(*[int(s[0]) for s in schedule])
        ec = (ctypes.c_double * n)(*[float(s[1]) for s in schedule])
        ms = (ctypes.c_int * n)(*[int(s[2]) for s in schedule])
        nz = (ctypes.c_double * n)(*[float(s[3]) if len(s) > 3 else 0.0 for s in schedule])
        e = ctypes.c_double()
        self._chk(self.lib.sadmrg_solve(self.h, n, D, ec, ms, nz, ctypes.byref(e)))
        return e.value

    def solve_extrapolated(self, schedule):
        """The convergence scheme stage by stage with the discarded-weight
        extrapolation (sadmrg_solve_extrapolated).  Returns (E0, C1,
        [(D, w_disc, E(D))])."""
        n = len(schedule)
        D = (ctypes.c_int * n)(*[int(s[0]) for s in schedule])
        ec = (ctypes.c_double * n)(*[float(s[1]) for s in schedule])
        ms = (ctypes.c_int * n)(*[int(s[2]) for s in schedule])
        nz = (ctypes.c_double * n)(*[float(s[3]) if len(s) > 3 else 0.0 for s in schedule])
        pts = (ctypes.c_double * (3 * n))()
        e0, c1 = ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.sadmrg_solve_extrapolated(self.h, n, D, ec, ms, nz, pts, ctypes.byref(e0),
                                                     ctypes.byref(c1)))
        points = [(int(pts[3 * i]), pts[3 * i + 1], pts[3 * i + 2]) for i in range(n)]
        return e0.value, c1.value, points

    def dmrgscf(self, orb_irrep, cls, h, eri, schedule, e_nuc=0.0, grad_tol=1e-6, max_iter=30, max_step=0.5,
                U0=None):
        """sadmrg_dmrgscf on this active-space solver.  Returns (E, U, history
        [(E, |g|)], iterations)."""
        Lt = len(cls)
        irr = np.ascontiguousarray(orb_irrep, dtype=np.int32)
        cl = np.ascontiguousarray(cls, dtype=np.int32)
        h = np.ascontiguousarray(h, dtype=np.float64)
        eri = np.ascontiguousarray(eri, dtype=np.float64)
        n = len(schedule)
        D = (ctypes.c_int * n)(*[int(s[0]) for s in schedule])
        ec = (ctypes.c_double * n)(*[float(s[1]) for s in schedule])
        ms = (ctypes.c_int * n)(*[int(s[2]) for s in schedule])
        nz = (ctypes.c_double * n)(*[float(s[3]) if len(s) > 3 else 0.0 for s in schedule])
        U = np.eye(Lt) if U0 is None else np.array(U0, dtype=np.float64)
        U = np.ascontiguousarray(U)
        hist = np.zeros(2 * max_iter)
        it, e = ctypes.c_int(), ctypes.c_double()
        ip = ctypes.POINTER(ctypes.c_int)
        self._chk(self.lib.sadmrg_dmrgscf(self.h, Lt, irr.ctypes.data_as(ip), cl.ctypes.data_as(ip), float(e_nuc),
                                          _dptr(h), _dptr(eri), n, D, ec, ms, nz, float(grad_tol), int(max_iter),
                                          float(max_step), _dptr(U), _dptr(hist), ctypes.byref(it),
                                          ctypes.byref(e)))
        k = it.value
        return e.value, U, [(hist[2 * i], hist[2 * i + 1]) for i in range(k)], k

    def push_excitation(self, eta):
        """Keep the current MPS as a lower state with weight eta (sadmrg_push_excitation)."""
        self._chk(self.lib.sadmrg_push_excitation(self.h, float(eta)))

    def clear_excitations(self):
        self._chk(self.lib.sadmrg_clear_excitations(self.h))

    def energy(self):
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.sadmrg_get_energy(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def trace(self):
        n = ctypes.c_int(0)
        self._chk(self.lib.sadmrg_get_trace(self.h, None, ctypes.byref(n)))
        out = np.zeros(n.value)
        self._chk(self.lib.sadmrg_get_trace(self.h, _dptr(out), ctypes.byref(n)))
        return out

    # ---- MPS exchange
    def mps_import(self, blob: bytes):
        buf = ctypes.create_string_buffer(blob, len(blob))
        self._chk(self.lib.sadmrg_mps_import(self.h, buf, len(blob)))

    def mps_export(self) -> bytes:
        n = ctypes.c_size_t(0)
        self._chk(self.lib.sadmrg_mps_export(self.h, None, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        self._chk(self.lib.sadmrg_mps_export(self.h, buf, ctypes.byref(n)))
        return buf.raw[: n.value]

    # ---- single-step hooks
    def prepare_step(self):
        self._chk(self.lib.sadmrg_prepare_step(self.h))

    def advance(self, D, n):
        e = ctypes.c_double()
        self._chk(self.lib.sadmrg_advance(self.h, int(D), int(n), ctypes.byref(e)))
        return e.value

    def task_shapes(self):
        n = ctypes.c_int64(0)
        self._chk(self.lib.sadmrg_debug_task_shapes(self.h, None, ctypes.byref(n)))
        out = np.zeros((n.value, 5), dtype=np.int32)
        self._chk(self.lib.sadmrg_debug_task_shapes(self.h, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                                    ctypes.byref(n)))
        return out

    def psi_layout(self):
        ns = ctypes.c_int(0)
        n = ctypes.c_int64(0)
        self._chk(self.lib.sadmrg_psi_layout(self.h, ctypes.byref(ns), None, ctypes.byref(n)))
        desc = np.zeros((ns.value, 6), dtype=np.int64)
        self._chk(self.lib.sadmrg_psi_layout(self.h, ctypes.byref(ns),
                                             desc.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), ctypes.byref(n)))
        return desc, n.value

    def sigma(self, x):
        """Apply H_eff.  numpy in -> numpy out (host), torch CUDA tensor in -> tensor out."""
        if hasattr(x, "data_ptr") and getattr(x, "is_cuda", False):
            import torch
            xx = x.contiguous().to(torch.float64)
            y = torch.empty_like(xx)
            self._chk(self.lib.sadmrg_sigma(self.h, ctypes.c_void_p(xx.data_ptr()), ctypes.c_void_p(y.data_ptr()), 1))
            return y
        xx = np.ascontiguousarray(x, dtype=np.float64)
        y = np.zeros_like(xx)
        self._chk(self.lib.sadmrg_sigma(self.h, xx.ctypes.data_as(ctypes.c_void_p),
                                        y.ctypes.data_as(ctypes.c_void_p), 0))
        return y

    def sigma_noalloc(self, x, y=None):
        """sadmrg_sigma_noalloc: x (and y) are torch CUDA float64 tensors of the
        prepared step's length; the library allocates no device memory."""
        if y is None:
            import torch
            y = torch.empty_like(x)
        if not (getattr(x, "is_cuda", False) and getattr(y, "is_cuda", False)):
            raise ValueError("sigma_noalloc takes device tensors")
        self._chk(self.lib.sadmrg_sigma_noalloc(self.h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr())))
        return y

    def heff_diagonal(self):
        _, n = self.psi_layout()
        d = np.zeros(n)
        self._chk(self.lib.sadmrg_heff_diagonal(self.h, d.ctypes.data_as(ctypes.c_void_p), 0))
        return d

    def guess(self):
        """Initial Davidson vector of the prepared step (host copy)."""
        _, n = self.psi_layout()
        d = np.zeros(n)
        self._chk(self.lib.sadmrg_debug_guess(self.h, d.ctypes.data_as(ctypes.c_void_p), 0))
        return d

    def plan_stats(self):
        """((pieces, workgroups, cut tiles) of pass 1, same of pass 2)."""
        out = (ctypes.c_int64 * 6)()
        self._chk(self.lib.sadmrg_debug_plan_stats(self.h, out))
        return tuple(out[:3]), tuple(out[3:])

    def sigma_counters(self):
        f, b = ctypes.c_double(), ctypes.c_double()
        t = ctypes.c_int64()
        self._chk(self.lib.sadmrg_sigma_counters(self.h, ctypes.byref(f), ctypes.byref(b), ctypes.byref(t)))
        return f.value, b.value, t.value

    def stats(self):
        ts, tm, fs, tb = ctypes.c_double(), ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        ns = ctypes.c_int64()
        self._chk(self.lib.sadmrg_stats(self.h, ctypes.byref(ts), ctypes.byref(ns), ctypes.byref(tm),
                                        ctypes.byref(fs), ctypes.byref(tb)))
        bs, me = ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.sadmrg_stats_bytes(self.h, ctypes.byref(bs), ctypes.byref(me)))
        p1 = (ctypes.c_double * 4)()
        p2 = (ctypes.c_double * 4)()
        self._chk(self.lib.sadmrg_stats_passes(self.h, p1, p2))
        out = {"t_sigma": ts.value, "n_sigma": ns.value, "t_micro": tm.value, "flops_sigma": fs.value,
               "t_blocking": tb.value, "bytes_sigma": bs.value, "max_enlarged_bytes": me.value}
        for name, arr in (("pass1", p1), ("pass2", p2)):
            out[name] = {"t": arr[0], "flops": arr[1], "bytes": arr[2], "launches": int(arr[3])}
        t32, n32, f32 = ctypes.c_double(), ctypes.c_int64(), ctypes.c_double()
        self._chk(self.lib.sadmrg_stats_mixed(self.h, ctypes.byref(t32), ctypes.byref(n32), ctypes.byref(f32)))
        out["fp32"] = {"t": t32.value, "calls": n32.value, "flops": f32.value}
        ph = (ctypes.c_double * 7)()
        self._chk(self.lib.sadmrg_stats_phases(self.h, ph))
        out["phases"] = dict(zip(("enlarge", "tasks", "plan", "diag", "guess", "svd", "renorm"), list(ph)))
        return out

    def rdm(self, two_body: bool = True):
        """(gamma [L,L], Gamma^A [L,L,L,L] or None, E) at the current two-site centre."""
        L = self.L
        g1 = np.zeros((L, L))
        g2 = np.zeros((L, L, L, L)) if two_body else None
        e = ctypes.c_double()
        self._chk(self.lib.sadmrg_rdm(self.h, _dptr(g1), _dptr(g2) if two_body else None, ctypes.byref(e)))
        return g1, g2, e.value

    def calc2dm(self, layout: int = 0):
        """The paper's calc2DM outputs from one reverse pass:
        (Gamma^A [L]*4 in `layout` (0 paper, 1 chemist), Gamma^B (paper order,
        multiplet average), gamma, <S^2>, E)."""
        L = self.L
        ga, gb, g1 = np.zeros((L,) * 4), np.zeros((L,) * 4), np.zeros((L, L))
        s2, e = ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.sadmrg_calc2dm(self.h, _dptr(ga), _dptr(gb), int(layout), _dptr(g1), ctypes.byref(s2),
                                          ctypes.byref(e)))
        return ga, gb, g1, s2.value, e.value

    def s2(self) -> float:
        v = ctypes.c_double()
        self._chk(self.lib.sadmrg_get_s2(self.h, ctypes.byref(v)))
        return v.value

    def autotune(self, reps: int = 5):
        """Tune the sigma launch shape on the prepared step (sadmrg_autotune).
        Returns ((gpc1, gpc2), [((g1, g2), ms), ...])."""
        a, b = ctypes.c_int(), ctypes.c_int()
        t = (ctypes.c_double * 36)()
        self._chk(self.lib.sadmrg_autotune(self.h, int(reps), ctypes.byref(a), ctypes.byref(b), t))
        return (a.value, b.value), [((int(t[2 * c]), int(t[2 * c + 1])), t[24 + c]) for c in range(12)]

    def set_launch_shape(self, gpc1: int, gpc2: int):
        self._chk(self.lib.sadmrg_set_launch_shape(self.h, int(gpc1), int(gpc2)))

    def set_contraction_order(self, mode: int):
        """0: each sigma product in the order with fewer flops; 1: fewer bytes
        streamed (sadmrg_set_contraction_order)."""
        self._chk(self.lib.sadmrg_set_contraction_order(self.h, int(mode)))

    def set_xcd_order(self, pass1: bool, pass2: bool):
        """XCD-grouped workgroup order of the two sigma passes (sadmrg_set_xcd_order)."""
        self._chk(self.lib.sadmrg_set_xcd_order(self.h, int(bool(pass1)), int(bool(pass2))))

    def set_enlarge_cache(self, on: bool):
        self._chk(self.lib.sadmrg_set_enlarge_cache(self.h, int(bool(on))))

    def set_precision(self, mode: int, mixed_tol: float = 1e-5):
        """0: FP64 sigma; 1 / 2: FP32 / BF16x3 sigma in Davidson, then one FP64
        Davidson step per micro-iteration (sadmrg_set_precision)."""
        self._chk(self.lib.sadmrg_set_precision(self.h, int(mode), float(mixed_tol)))

    def set_block_checkpoints(self, interval: int):
        """Keep renormalised blocks only every `interval` bonds and rebuild the
        others when needed (sadmrg_set_block_checkpoints); 0 keeps all."""
        self._chk(self.lib.sadmrg_set_block_checkpoints(self.h, int(interval)))

    def stats_blocks(self):
        """(blocks rebuilt, rebuild seconds, largest block bytes held, blocks held now)."""
        n, t, b, h = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double(), ctypes.c_int()
        self._chk(self.lib.sadmrg_stats_blocks(self.h, ctypes.byref(n), ctypes.byref(t), ctypes.byref(b),
                                               ctypes.byref(h)))
        return {"rebuilt": n.value, "seconds": t.value, "max_bytes": b.value, "held": h.value}

    def set_davidson_graph(self, replays: int):
        """Davidson iterations replayed from a recorded HIP graph, `replays`
        per host check; 0 = host-driven (sadmrg_set_davidson_graph)."""
        self._chk(self.lib.sadmrg_set_davidson_graph(self.h, int(replays)))

    def stats_graph(self):
        """Counters of the recorded Davidson iterations (sadmrg_stats_graph)."""
        t, tr, f = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        n, r, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._chk(self.lib.sadmrg_stats_graph(self.h, ctypes.byref(t), ctypes.byref(tr), ctypes.byref(f),
                                              ctypes.byref(n), ctypes.byref(r), ctypes.byref(c)))
        return {"seconds": t.value, "record_seconds": tr.value, "sigma_flops": f.value, "sigma_calls": n.value,
                "replays": r.value, "records": c.value}

    def set_renorm_precision(self, mode: int):
        """0 FP64, 1 FP32, 2 BF16x3 renormalisation products (sadmrg_set_renorm_precision)."""
        self._chk(self.lib.sadmrg_set_renorm_precision(self.h, int(mode)))

    def set_refinement_tol(self, tol: float):
        """Residual target of the FP64 refinement (sadmrg_set_refinement_tol)."""
        self._chk(self.lib.sadmrg_set_refinement_tol(self.h, float(tol)))

    def set_refinement(self, steps: int):
        """FP64 Davidson steps after the reduced-precision phase (modes 1, 2)."""
        self._chk(self.lib.sadmrg_set_refinement(self.h, int(steps)))

    def copy_probe(self, n: int, reps: int = 5) -> float:
        """Mean seconds of the library's plain streaming-copy kernel over n doubles."""
        s = ctypes.c_double()
        self._chk(self.lib.sadmrg_debug_copy_probe(self.h, int(n), int(reps), ctypes.byref(s)))
        return s.value

    def set_method_counter(self, on: bool):
        self._chk(self.lib.sadmrg_set_method_counter(self.h, int(bool(on))))

    def stats_method(self):
        """(method flops, performed flops) of the counted FP64 sigma calls and
        the prepared step's method flops (sadmrg_stats_method)."""
        a, b, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.sadmrg_stats_method(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
        return a.value, b.value, c.value

    def gemm_probe(self, nprod: int, K: int, reps: int = 5):
        """(seconds per launch, exact bytes per launch) of the reference GEMM."""
        s, b = ctypes.c_double(), ctypes.c_double()
        self._chk(self.lib.sadmrg_debug_gemm_probe(self.h, int(nprod), int(K), int(reps), ctypes.byref(s),
                                                   ctypes.byref(b)))
        return s.value, b.value

    def stats_reset(self):
        self._chk(self.lib.sadmrg_stats_reset(self.h))


def fit_discarded_weight(points, lib_path: str | None = None):
    """E0, C1 of the line E = E0 + C1 w through (w_disc, E) pairs
    (sadmrg_extrapolate: section "Extrapolation")."""
    pts = [(float(w), float(e)) for w, e in points]
    if not pts:
        raise ValueError("no (w_disc, E) pairs")
    lib = load_library(lib_path)
    n = len(pts)
    w = (ctypes.c_double * n)(*[p[0] for p in pts])
    e = (ctypes.c_double * n)(*[p[1] for p in pts])
    e0, c1 = ctypes.c_double(), ctypes.c_double()
    rc = lib.sadmrg_extrapolate(n, w, e, ctypes.byref(e0), ctypes.byref(c1))
    if rc != 0:
        raise SadmrgError(rc, "bad (w, E) pairs")
    return e0.value, c1.value


def rotate_integrals(R, h, eri, lib_path: str | None = None):
    """(R^T h R, eri with R on every index) (sadmrg_rotate_integrals)."""
    lib = load_library(lib_path)
    R, h, eri = (np.ascontiguousarray(a, dtype=np.float64) for a in (R, h, eri))
    L = h.shape[0]
    h2, e2 = np.zeros_like(h), np.zeros_like(eri)
    rc = lib.sadmrg_rotate_integrals(L, _dptr(R), _dptr(h), _dptr(eri), _dptr(h2), _dptr(e2))
    if rc != 0:
        raise SadmrgError(rc, "sadmrg_rotate_integrals failed")
    return h2, e2


def rotation(kappa, lib_path: str | None = None):
    """exp(kappa) of an antisymmetric matrix (sadmrg_rotation)."""
    lib = load_library(lib_path)
    k = np.ascontiguousarray(kappa, dtype=np.float64)
    R = np.zeros_like(k)
    rc = lib.sadmrg_rotation(k.shape[0], _dptr(k), _dptr(R))
    if rc != 0:
        raise SadmrgError(rc, "sadmrg_rotation failed")
    return R


def orbital_derivatives(h, eri, D, d, pairs, hessian=True, lib_path: str | None = None):
    """(gradient, Hessian or None, generalised Fock) of E over `pairs` with
    the RDMs fixed (sadmrg_orbital_derivatives)."""
    lib = load_library(lib_path)
    h, eri, D, d = (np.ascontiguousarray(a, dtype=np.float64) for a in (h, eri, D, d))
    L = h.shape[0]
    n = len(pairs)
    pr = np.ascontiguousarray(np.array(pairs, dtype=np.int32).reshape(-1))
    g = np.zeros(max(n, 1))
    H = np.zeros((n, n)) if hessian else None
    F = np.zeros((L, L))
    rc = lib.sadmrg_orbital_derivatives(L, _dptr(h), _dptr(eri), _dptr(D), _dptr(d), n,
                                        pr.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(g),
                                        _dptr(H) if hessian else None, _dptr(F))
    if rc != 0:
        raise SadmrgError(rc, "sadmrg_orbital_derivatives failed")
    return g[:n], H, F


def device_memory(device: int = 0, lib_path: str | None = None):
    """(free, total) bytes of device memory (sadmrg_device_memory)."""
    lib = load_library(lib_path)
    f, t = ctypes.c_size_t(), ctypes.c_size_t()
    rc = lib.sadmrg_device_memory(int(device), ctypes.byref(f), ctypes.byref(t))
    if rc != 0:
        raise SadmrgError(rc, "sadmrg_device_memory failed")
    return f.value, t.value


def batch_sweep(solvers, D):
    """One lockstep macro-iteration of several solvers (sadmrg_batch_sweep).

    solvers: SaDMRG objects sharing one library, device, stream and precision;
    D: one bond dimension per solver (or a single int for all).
    Returns (e_min list, stats dict, rc)."""
    solvers = list(solvers)
    n = len(solvers)
    if n == 0:
        raise ValueError("empty batch")
    lib = solvers[0].lib
    if any(s.lib is not lib for s in solvers):
        raise ValueError("solvers of different libraries")
    Ds = [int(D)] * n if np.isscalar(D) else [int(d) for d in D]
    if len(Ds) != n:
        raise ValueError("one D per solver")
    hs = (ctypes.c_void_p * n)(*[s.h for s in solvers])
    dd = (ctypes.c_int * n)(*Ds)
    em = (ctypes.c_double * n)()
    st = (ctypes.c_double * 10)()
    rc = lib.sadmrg_batch_sweep(hs, n, dd, em, st)
    if rc < 0:
        msg = lib.sadmrg_last_error(solvers[0].h)
        raise SadmrgError(rc, msg.decode() if msg else "")
    stats = {"t_sigma": st[0], "flops_sigma": st[1], "n_sigma": int(st[2]),
             "t_sigma32": st[3], "flops_sigma32": st[4], "n_sigma32": int(st[5]),
             "wall": {"prepare": st[6], "davidson": st[7], "refine": st[8], "finish": st[9]}}
    return list(em), stats, rc


def debug_coupling(which: int, args, lib_path: str | None = None) -> float:
    lib = load_library(lib_path)
    a = (ctypes.c_int * len(args))(*[int(v) for v in args])
    out = ctypes.c_double()
    rc = lib.sadmrg_debug_coupling(int(which), a, ctypes.byref(out))
    if rc != 0:
        raise SadmrgError(rc, "bad coupling request")
    return out.value
