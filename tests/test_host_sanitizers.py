"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

Every source under paper_2212_09664_amd/csrc is compiled with the sanitizers
on its host half only (each -fsanitize flag behind -Xarch_host; the device
half is built as usual for gfx950) and linked with tests/host_checks.cpp,
which drives the entry points that make no GPU call: context creation over a
grid of shapes, the parameter checks, null arguments, calls before a problem
is bound, and the warm-start network's host bookkeeping.  Runs on the CPU."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-g"]


def _run(cmd):
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"{' '.join(cmd)}\n{res.stderr[-4000:]}")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_host_entry_points_under_sanitizers(tmp_path):
    from paper_2212_09664_amd import build
    flags = [f for f in build.FLAGS if f != "-O3"] + ["-O1"]
    csrc = os.path.join(ROOT, "paper_2212_09664_amd", "csrc")
    jobs = [([HIPCC, *flags, *SAN, "-c", os.path.join(csrc, s), "-o", str(tmp_path / (s + ".o"))])
            for s in build.SOURCES]
    jobs.append([HIPCC, "--offload-host-only", "-O1", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"),
                 "-c", os.path.join(ROOT, "tests", "host_checks.cpp"), "-o", str(tmp_path / "host_checks.o")])
    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(_run, jobs))
    exe = str(tmp_path / "host_checks")
    objs = [str(tmp_path / (s + ".o")) for s in build.SOURCES] + [str(tmp_path / "host_checks.o")]
    _run([HIPCC, "--offload-arch=gfx950", *SAN, *objs, "-o", exe])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout[-2000:] + res.stderr[-4000:]
    assert "host checks passed" in res.stdout
