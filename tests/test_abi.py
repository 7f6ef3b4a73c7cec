"""The C ABI without a GPU: the library loads, exports every function that
include/mirve.h declares, and its host-only entry points (defaults, version,
workspace query and configuration checks) behave as documented.  No call
here launches a kernel or touches device memory."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mirve.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(rve_\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_2508_07424_amd import mirve
    if not os.path.exists(mirve.LIB_PATH):
        pytest.fail("libmirve.so is not built (python -m paper_2508_07424_amd.build)")
    return mirve


def test_header_parses():
    names = declared_functions()
    assert len(names) >= 25
    for core in ("rve_create", "rve_set_microstructure", "rve_step_dissipation",
                 "rve_effective_toughness", "rve_query_workspace", "rve_last_error"):
        assert core in names


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    so = C.CDLL(lib.LIB_PATH)
    missing = [n for n in names if not hasattr(so, n)]
    assert not missing, missing
    # the dynamic symbol table agrees, and the binding covers the header
    out = subprocess.run(["nm", "-D", "--defined-only", lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\bT (rve_\w+)$", out, flags=re.M))
    assert set(names) <= exported
    assert set(names) == set(lib.EXPORTS)


def test_struct_layouts_match_header(lib, tmp_path):
    """The binding's ctypes structures have the sizes and field offsets that
    a C compiler gives the header's structures."""
    structs = {"rve_config": lib.rve_config, "rve_phase": lib.rve_phase,
               "rve_step_info": lib.rve_step_info}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "mirve.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append('printf("%s %%zu\\n", sizeof(%s));' % (name, name))
        for fname, _ in cls._fields_:
            lines.append('printf("%s.%s %%zu\\n", offsetof(%s, %s));' % (name, fname, name, fname))
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    got = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(got[name]) == C.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(got[name + "." + fname]) == getattr(cls, fname).offset, (name, fname)


def test_version_and_defaults(lib):
    so = lib.lib
    assert b"gfx950" in so.rve_version()
    cfg = lib.rve_config()
    assert so.rve_default_config(C.byref(cfg)) == lib.RVE_OK
    assert cfg.dim == 2 and tuple(cfg.n) == (64, 64, 1) and cfg.batch == 1
    assert cfg.k_res == 1e-6 and cfg.f[1] == 1.0 and cfg.split == lib.RVE_SPLIT_NONE
    assert cfg.graphs == 1 and cfg.streaming == -1
    # tolerances 0: the library resolves them per precision at rve_create
    assert cfg.tol == cfg.tol_cg == cfg.tol_pcg == cfg.tol_al == 0.0
    assert cfg.max_halvings == 8 and cfg.stall_window == 0
    assert so.rve_default_config(None) == lib.RVE_EINVAL


def _query(lib, **kw):
    cfg = lib.make_config(**kw)
    nb = C.c_size_t(0)
    rc = lib.lib.rve_query_workspace(C.byref(cfg), C.byref(nb))
    return rc, nb.value


def test_workspace_query(lib):
    rc, b1 = _query(lib, n=(64, 64), precision=lib.RVE_PREC_FP64)
    assert rc == lib.RVE_OK and b1 > 0
    # footprint grows with the batch and halves (roughly) in mixed precision
    rc, b9 = _query(lib, n=(64, 64), precision=lib.RVE_PREC_FP64, batch=9)
    assert rc == lib.RVE_OK and 8 * b1 < b9 < 10 * b1
    rc, bm = _query(lib, n=(256, 256), precision=lib.RVE_PREC_MIXED)
    rc2, bd = _query(lib, n=(256, 256), precision=lib.RVE_PREC_FP64)
    assert rc == rc2 == lib.RVE_OK and 0.4 * bd < bm < 0.7 * bd
    # 3D and 7-smooth sizes are accepted
    assert _query(lib, n=(32, 32, 32), f=(0, 0, 1, 0, 0, 0))[0] == lib.RVE_OK
    assert _query(lib, n=(96, 80))[0] == lib.RVE_OK
    assert _query(lib, n=(98, 70))[0] == lib.RVE_OK


@pytest.mark.parametrize("bad", [
    {"dim": 4}, {"n": (1, 64)}, {"n": (64, 2048)}, {"h": 0.0}, {"ell": -1.0},
    {"tol_cg": -1e-8}, {"tol": float("nan")}, {"max_cg": 0}, {"max_halvings": 13},
    {"max_halvings": -1}, {"stall_window": -1}, {"batch": 0}, {"batch": 5000}, {"anderson_depth": 9},
    {"f": (0, 0, 0)}, {"n": (97, 64)},   # 97 is prime: no FFT factorisation
    {"streaming": 2}, {"streaming": -2}, {"graphs": 2}, {"ell": float("nan")}, {"k": float("inf")},
    {"h": float("inf")},
])
def test_invalid_configs_are_rejected(lib, bad):
    kw = {"n": (64, 64)}
    kw.update(bad)
    rc, _ = _query(lib, **kw)
    assert rc == lib.RVE_EINVAL
    msg = lib.lib.rve_last_error(None)
    assert msg and len(msg) > 3


def test_create_rejects_without_workspace(lib):
    cfg = lib.make_config(n=(64, 64))
    h = C.c_void_p()
    so = lib.lib
    assert so.rve_create(C.byref(cfg), None, 0, None, C.byref(h)) == lib.RVE_EINVAL
    assert not h.value
    assert so.rve_create(C.byref(cfg), C.c_void_p(256), 16, None, C.byref(h)) == lib.RVE_ENOSPC
    assert so.rve_create(C.byref(cfg), C.c_void_p(4096 + 8), 1 << 40, None, C.byref(h)) == lib.RVE_EINVAL
