"""The C-ABI library loads on the host and exports every declared symbol;
argument checking and quick returns need no device."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_2305_19917_amd as rs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "redsea.h")).read()
    return sorted(set(re.findall(r"\b(redsea_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert _declared() == sorted(rs.EXPORTS)


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", rs.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (redsea_\w+)", out))
    for name in _declared():
        assert name in exported, name
        assert getattr(rs.lib(), name) is not None


def test_version_and_status_strings():
    assert re.match(r"^\d+\.\d+\.\d+\+[0-9a-f]{12}$", rs.version())
    from paper_2305_19917_amd import build
    assert rs.version().endswith(build.build_id())
    assert rs.status_string(0) == "success"
    assert "invalid" in rs.status_string(-3)
    for code in range(1, 6):
        assert rs.status_string(code) != "unknown status"


def _trsm_raw(**kw):
    args = dict(dtype=0, side=0, uplo=0, trans=0, diag=0, m=4, n=3, alpha=1.0, A=8, lda=4, B=8,
                ldb=4)
    args.update(kw)
    L = rs.lib()
    return L.redsea_trsm(args["dtype"], args["side"], args["uplo"], args["trans"], args["diag"],
                         args["m"], args["n"], args["alpha"], args["A"], args["lda"], args["B"],
                         args["ldb"], None, None)


@pytest.mark.parametrize("kw,code", [
    (dict(dtype=7), -1), (dict(side=2), -2), (dict(uplo=-1), -3), (dict(trans=3), -4),
    (dict(diag=2), -5), (dict(m=-1), -6), (dict(n=-2), -7), (dict(lda=3), -10),
    (dict(ldb=3), -12), (dict(A=None), -9), (dict(B=None), -11),
    (dict(side=1, lda=2), -10),
])
def test_argument_errors(kw, code):
    assert _trsm_raw(**kw) == code


def test_quick_returns_touch_nothing():
    # NULL pointers are fine when there is nothing to do
    assert _trsm_raw(m=0, A=None, B=None) == 0
    assert _trsm_raw(n=0, A=None, B=None) == 0


def test_bad_options():
    L = rs.lib()
    for opts in (rs.Opts(9, 0, 0), rs.Opts(0, 48, 0), rs.Opts(0, 0, 7)):
        assert L.redsea_trsm(0, 0, 0, 0, 0, 4, 3, 1.0, 8, 4, 8, 4, ctypes.byref(opts), None) == -13


def test_batched_argument_errors():
    L = rs.lib()
    i64 = ctypes.c_int64
    m = (i64 * 1)(4)
    n = (i64 * 1)(3)
    lda = (i64 * 1)(2)
    ldb = (i64 * 1)(4)
    ptrs = (ctypes.c_void_p * 1)(8)
    assert L.redsea_trsm_batched(0, 0, 0, 0, 0, -1, m, n, 1.0, ptrs, lda, ptrs, ldb, 8, None,
                                 None) == -6
    assert L.redsea_trsm_batched(0, 0, 0, 0, 0, 0, None, None, 1.0, None, None, None, None, None,
                                 None, None) == 0
    assert L.redsea_trsm_batched(0, 0, 0, 0, 0, 1, m, n, 1.0, ptrs, lda, ptrs, ldb, 8, None,
                                 None) == -11


@pytest.mark.parametrize("args,code", [
    ((7, 0, 4, 8, 4, 0, 8), -1), ((0, 2, 4, 8, 4, 0, 8), -2), ((0, 0, -1, 8, 4, 0, 8), -3),
    ((0, 0, 4, 8, 3, 0, 8), -5), ((0, 0, 4, 8, 4, 48, 8), -6), ((0, 0, 4, 8, 4, 256, 8), -6),
    ((0, 0, 4, 8, 4, 0, None), -7), ((0, 0, 4, None, 4, 0, 8), -4),
])
def test_potrf_argument_errors(args, code):
    # checked before any device work, so no GPU is needed
    assert rs.lib().redsea_potrf(*args, None) == code


def test_schedule_argument_errors():
    L = rs.lib()
    assert L.redsea_schedule(5, 10, 16, None, 0) == -1
    assert L.redsea_schedule(1, -1, 16, None, 0) == -2
    assert L.redsea_schedule(1, 10, 0, None, 0) == -3
    assert L.redsea_schedule(1, 10, 16, None, 5) == -4
    assert L.redsea_schedule(1, 0, 16, None, 0) == 0


def test_picker_outside_trained_shapes_takes_default_schedule():
    """Outside the orders and widths the network was trained on, the host
    picker returns the default schedule (recursive, native precision, nb 256
    above order 128, else 128) and reports no confidence; inside, it returns
    a valid candidate."""
    L = rs.lib()
    conf = ctypes.c_int(7)
    var, nb, prec = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    # the stored network was trained on orders 65 .. 32445 and widths 1 .. 16238
    for dtype, n, nrhs, want_nb in [(0, 65536, 1024, 256), (1, 4096, 65536, 256),
                                    (0, 100, 100000, 128), (0, 32, 4, 128)]:
        c = L.redsea_pick(dtype, n, nrhs, 0.0, ctypes.byref(conf))
        assert conf.value == 0
        assert L.redsea_candidate(c, ctypes.byref(var), ctypes.byref(nb), ctypes.byref(prec)) == 0
        assert (var.value, nb.value, prec.value) == (1, want_nb, 1), (n, nrhs, c)
    c = L.redsea_pick(0, 2000, 300, 9000.0, ctypes.byref(conf))
    assert 0 <= c < 45


def _consumer_source():
    names = _declared()
    fns = ",\n    ".join("(fp)%s" % n for n in names)
    return """#include "redsea.h"
#include <stdio.h>
#include <string.h>
typedef void (*fp)(void);
static fp every_entry[] = {
    %s
};
int main(void) {
    redsea_opts o = {REDSEA_VARIANT_RECURSIVE, 256, REDSEA_PREC_NATIVE, 0.0, 0};
    redsea_mixed_stats st;
    memset(&st, 0, sizeof st);
    (void)o;
    printf("%%s %%s %%d\\n", redsea_version(), redsea_status_string(REDSEA_OK),
           (int)(sizeof every_entry / sizeof every_entry[0]));
    return 0;
}
""" % fns


@pytest.mark.parametrize("compiler,std,ext", [("gcc", "-std=c11", "c"), ("g++", "-std=c++17", "cpp")])
def test_header_compiles_standalone_and_links(tmp_path, compiler, std, ext):
    """A C (or C++) client that includes only redsea.h builds warning-free,
    takes the address of every declared entry point, links against
    libredsea.so and runs (no device call)."""
    src = tmp_path / ("consumer." + ext)
    src.write_text(_consumer_source())
    exe = tmp_path / "consumer"
    libdir = os.path.dirname(rs.LIB_PATH)
    subprocess.run([compiler, std, "-Wall", "-Wextra", "-Werror", "-pedantic",
                    "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                    "-L", libdir, "-lredsea", "-Wl,-rpath," + libdir],
                   check=True, capture_output=True, text=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()
    assert out[0] == rs.version() and out[1] == "success"
    assert int(out[2]) == len(_declared())


def test_batched_tune_argument_errors():
    L = rs.lib()
    i64 = ctypes.c_int64
    k = (i64 * 1)(10)
    r = (i64 * 1)(3)
    best = ctypes.c_int(0)
    assert L.redsea_batched_tune(5, 0, 1, k, r, 1, None, ctypes.byref(best)) == -1
    assert L.redsea_batched_tune(0, 3, 1, k, r, 1, None, ctypes.byref(best)) == -2
    assert L.redsea_batched_tune(0, 0, -1, k, r, 1, None, ctypes.byref(best)) == -3
    assert L.redsea_batched_tune(0, 0, 1, None, r, 1, None, ctypes.byref(best)) == -4
    assert L.redsea_batched_tune(0, 0, 1, k, r, 0, None, ctypes.byref(best)) == -6
    assert L.redsea_batched_tune(0, 0, 1, k, r, 1, None, None) == -8
    assert L.redsea_batched_tune(0, 0, 0, None, None, 1, None, ctypes.byref(best)) == 0
    assert best.value == 1


def test_potrf_binding_refuses_host_tensors():
    # the library writes info and the factor through device pointers: the
    # binding refuses host tensors before any call
    torch = pytest.importorskip("torch")
    A = torch.zeros((4, 4), dtype=torch.float64).t()
    with pytest.raises(ValueError):
        rs.potrf(A)
