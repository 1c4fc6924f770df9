"""The engine's host code under ThreadSanitizer and AddressSanitizer.

engine.cpp, su2.cpp, scf.cpp and pool.cpp (the device-memory pools) are
compiled with g++ against a CPU stand-in for the device layer
(tests/cpu_emu/kernels_emu.cpp: host memory, synchronous launches with the
record semantics of kernels.h) into a test executable that is never loaded by
the Python binding.  The driver (tests/cpu_emu/driver.cpp) runs the batched
sweep pattern -- five contexts in lockstep, whose preparation and update run
on the library's host worker threads, in FP64, then mixed precision with
checkpointed blocks, then separate sweeps and the energy adjoint -- and
checks that lockstep and separate sweeps agree.  The AddressSanitizer run
then injects device errors (a gather and a GEMM launch, in a batch and in a
single sweep), each of which must come back as an error of the call and
leave the contexts and their memory pools usable (a buffer released while
such an error unwound once went back to no pool and was freed twice), and
compares the block-Jacobi decomposition of wide sectors with the
one-workgroup decomposition over six micro-iterations of a larger problem;
both are left out of the slower ThreadSanitizer run.  Both sanitizer runs
must end cleanly with no report.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1312_2415_amd", "csrc")
SOURCES = [os.path.join(CSRC, f) for f in ("engine.cpp", "su2.cpp", "scf.cpp", "pool.cpp")] + [
    os.path.join(HERE, "cpu_emu", "kernels_emu.cpp"), os.path.join(HERE, "cpu_emu", "driver.cpp")]
OUT = os.path.join(ROOT, "_build_emu")
VARIANTS = {
    "tsan": (["-fsanitize=thread"], {"TSAN_OPTIONS": "halt_on_error=1"}, "ThreadSanitizer",
             ["--no-block", "--no-inject"]),
    "asan": (["-fsanitize=address", "-fno-omit-frame-pointer"], {"ASAN_OPTIONS": "detect_leaks=1"},
             "Sanitizer", []),
}


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_engine_host_code_is_clean_under_sanitizers():
    os.makedirs(OUT, exist_ok=True)
    builds = {}
    for name, (flags, _, _, _) in VARIANTS.items():
        exe = os.path.join(OUT, f"driver_{name}")
        cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", *flags, f"-I{CSRC}", *SOURCES, "-o", exe]
        builds[name] = (exe, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
    for name, (exe, proc) in builds.items():
        out, _ = proc.communicate(timeout=900)
        assert proc.returncode == 0, f"{name} build failed:\n{out[-4000:]}"
    runs = {}
    for name, (exe, _) in builds.items():
        env = dict(os.environ, **VARIANTS[name][1])
        runs[name] = subprocess.Popen([exe, *VARIANTS[name][3]], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, env=env)
    for name, proc in runs.items():
        out, _ = proc.communicate(timeout=900)
        print(out[-2000:])
        assert proc.returncode == 0, f"{name} run failed:\n{out[-6000:]}"
        assert VARIANTS[name][2] not in out, out[-6000:]
        assert "emulated batch" in out
        if not VARIANTS[name][3]:
            assert "block decomposition: 0 " not in out, out[-2000:]
