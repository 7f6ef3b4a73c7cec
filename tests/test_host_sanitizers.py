"""The host side of the library under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

Every source of the library is compiled for the host only (no device code),
with the sanitizers on the host pass, and linked with tests/host_driver.c,
which walks the entry points that need no GPU: defaults, version, workspace
queries of valid and invalid configurations, handle creation that fails
before any device work, and calls on a NULL handle.  A sanitizer report
fails the run."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2508_07424_amd", "csrc")
SOURCES = [("greenop.hip", ["-DMIRVE_REAL=double"], "greenop_f64.o"),
           ("greenop.hip", ["-DMIRVE_REAL=float"], "greenop_f32.o"),
           ("pointwise.hip", [], "pointwise.o"),
           ("newton.hip", [], "newton.o"),
           ("solver.hip", [], "solver.o")]
# the sanitizers apply to the host pass only (each flag after -Xarch_host)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g", "-O1"]


def _hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        pytest.skip("hipcc not available")
    return path


def test_host_entry_points_under_asan_ubsan(tmp_path):
    hipcc = _hipcc()
    base = [hipcc, "--offload-arch=gfx950", "--cuda-host-only", "-std=c++17", "-fPIC",
            "-I" + os.path.join(ROOT, "include")] + SAN

    def compile_one(item):
        src, extra, obj = item
        out = str(tmp_path / obj)
        r = subprocess.run(base + extra + ["-c", os.path.join(CSRC, src), "-o", out],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-4000:]
        return out

    with cf.ThreadPoolExecutor(max_workers=min(5, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    # A host-only object refers to the device code blob of its source by a
    # symbol; no kernel runs here (no device is visible), so an empty blob
    # stands in for each.
    names = set()
    for o in objs:
        r = subprocess.run(["nm", o], capture_output=True, text=True, check=True)
        names.update(l.split()[-1] for l in r.stdout.splitlines()
                     if l.split()[-1].startswith("__hip_fatbin_") and " U " in l)
    stub = tmp_path / "device_blobs.c"
    stub.write_text("".join("const char %s[64] __attribute__((aligned(4096))) = {0};\n" % n
                            for n in sorted(names)))
    r = subprocess.run(["gcc", "-c", "-fPIC", str(stub), "-o", str(tmp_path / "device_blobs.o")],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    objs.append(str(tmp_path / "device_blobs.o"))
    exe = str(tmp_path / "host_driver")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-x", "c", "-std=c11",
                        "-I" + os.path.join(ROOT, "include")] + SAN +
                       ["-c", os.path.join(ROOT, "tests", "host_driver.c"), "-o", exe + ".o"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    r = subprocess.run([hipcc, "--offload-arch=gfx950"] + SAN + [exe + ".o"] + objs +
                       ["-o", exe, "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx", "-lm",
                        "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ)
    # the HIP runtime's own start-up allocations are not the library's
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    env["HIP_VISIBLE_DEVICES"] = ""
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out, out[-4000:]
    assert "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and "host driver ok" in r.stdout, out[-4000:]
