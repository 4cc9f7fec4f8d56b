"""The C-ABI library loads, exports every symbol include/fgfrft.h declares, and
rejects bad arguments on the host (no GPU needed for any of these calls)."""
import ctypes
import os
import re

import pytest

from paper_2602_20870_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fgfrft.h")


def declared_symbols():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"FGFRFT_API\s+[\w\s\*]+?\b(fgfrft_\w+)\s*\(", text)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libfgfrft.so not built")
    return _lib.lib()


def test_header_declares_expected_entry_points():
    syms = declared_symbols()
    for name in ("fgfrft_plan", "fgfrft_update", "fgfrft_apply", "fgfrft_apply_operator", "fgfrft_grad",
                 "fgfrft_destroy", "fgfrft_strerror", "fgfrft_last_error"):
        assert name in syms


def test_every_declared_symbol_is_exported(L):
    syms = declared_symbols()
    assert set(syms) == set(_lib.SIGNATURES), "binding and header disagree"
    for name in syms:
        assert hasattr(L, name), name


def test_only_abi_symbols_are_exported(L):
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    fg = {s for s in exported if s.startswith("fgfrft_")}
    assert fg == set(declared_symbols())


def test_plan_bytes_validation(L):
    p, s = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.fgfrft_plan_bytes(0, 10, 1, 0, ctypes.byref(p), ctypes.byref(s)) == -1
    assert L.fgfrft_plan_bytes(64, 0, 1, 0, ctypes.byref(p), ctypes.byref(s)) == -1
    assert L.fgfrft_plan_bytes(64, 65, 1, 0, ctypes.byref(p), ctypes.byref(s)) == -1
    assert L.fgfrft_plan_bytes(64, 64, 0, 0, ctypes.byref(p), ctypes.byref(s)) == 0   # complex F up to L = 64
    assert L.fgfrft_plan_bytes(64, 65, 0, 0, ctypes.byref(p), ctypes.byref(s)) == -1
    assert L.fgfrft_plan_bytes(64, 10, 1, 3, ctypes.byref(p), ctypes.byref(s)) == -1   # no stack type 3
    assert L.fgfrft_plan_bytes(64, 10, 5, 0, ctypes.byref(p), ctypes.byref(s)) == -1
    assert L.fgfrft_plan_bytes(64, 10, 1, 0, ctypes.byref(p), ctypes.byref(s)) == 0
    N, Lt = 64, 10
    assert p.value >= Lt * N * N * 4 + N * N * 4
    assert s.value >= 4 * N * N * 8
    assert L.fgfrft_plan_bytes(64, 10, 0, 0, ctypes.byref(p), ctypes.byref(s)) == 0
    assert p.value >= Lt * N * N * 8 + N * N * 8


def test_null_and_small_arguments_are_rejected_on_host(L):
    h = ctypes.c_void_p()
    # NULL device pointers: rejected before any HIP call
    rc = L.fgfrft_plan(None, 16, 4, 1, 0, 0, 0.0, None, 0, None, 0, None, ctypes.byref(h))
    assert rc == -1 and not h.value
    assert b"NULL" in L.fgfrft_last_error()
    # an unknown operator form is rejected too (0: split, 1: standard)
    rc = L.fgfrft_plan(None, 16, 4, 1, 0, 2, 0.0, None, 0, None, 0, None, ctypes.byref(h))
    assert rc == -1 and b"form" in L.fgfrft_last_error()
    a = (ctypes.c_double * 2)(0.5, 0.25)
    assert L.fgfrft_update(None, a, 2, None, None, 0, None) == -1
    assert L.fgfrft_grad(None, a, 2, None, 0, 0, 4, None, None, None, None, 0, None) == -1
    assert L.fgfrft_apply_operator(None, 16, 1, 0, None, 0, 0, 4, None, 0, None, 0, None) == -1
    assert L.fgfrft_apply_operator(None, 0, 1, 0, None, 0, 0, 4, None, 0, None, 0, None) == -1
    assert L.fgfrft_update_workspace_bytes(None, 4) == 0
    # direct route: NULL plan, then no workspace size for a NULL plan
    assert L.fgfrft_apply_direct(None, None, 1, None, None, 0, 4, 4, None, 4, None, 0, None) == -1
    assert b"NULL plan" in L.fgfrft_last_error()
    assert L.fgfrft_apply_direct_workspace_bytes(None, 4, 4) == 0
    # grouped apply: NULL plan, and no workspace size for a NULL plan or a NULL count table
    bq = (ctypes.c_int * 2)(4, 3)
    ptrs = (ctypes.c_void_p * 2)(0x100000, 0x200000)
    assert L.fgfrft_apply_batched(None, a, 2, bq, ptrs, 0, ptrs, None, 0, None) == -1
    assert b"NULL plan" in L.fgfrft_last_error()
    assert L.fgfrft_apply_batched_workspace_bytes(None, 2, bq, 0) == 0
    # apply with device orders: NULL plan, and no workspace size for a NULL plan
    assert L.fgfrft_apply_dev(None, None, 1, None, 0, 0, 64, None, None, 0, None) == -1
    assert b"NULL plan" in L.fgfrft_last_error()
    assert L.fgfrft_apply_dev_workspace_bytes(None, 4, 64, 0, 0) == 0
    # traffic reference: NULL buffers, N not a multiple of 64, too many tiles (host-side refusals)
    assert L.fgfrft_probe_update_traffic(None, 64, 4, 1, None, None) == -1
    assert L.fgfrft_probe_update_traffic(0x100000, 96, 4, 1, 0x200000, None) == -1
    assert L.fgfrft_probe_update_traffic(0x100000, 64, 66, 1, 0x200000, None) == -1
    assert b"n_tiles" in L.fgfrft_last_error()



def test_misaligned_pointers_are_rejected_on_host(L):
    """Every argument but one pointer is valid; the misaligned pointer is refused before any HIP
    call (the fake addresses are never dereferenced)."""
    P = ctypes.c_void_p
    h = ctypes.c_void_p()
    pb, sb = ctypes.c_size_t(), ctypes.c_size_t()
    assert L.fgfrft_plan_bytes(64, 4, 1, 0, ctypes.byref(pb), ctypes.byref(sb)) == 0
    for F, pers, scr in ((0x100004, 0x200000, 0x300000), (0x100000, 0x200080, 0x300000),
                         (0x100000, 0x200000, 0x300010)):
        rc = L.fgfrft_plan(P(F), 64, 4, 1, 0, 0, 0.0, P(pers), pb.value, P(scr), sb.value, None, ctypes.byref(h))
        assert rc == -1 and not h.value and b"aligned" in L.fgfrft_last_error(), (F, pers, scr)
    N, n, B = 64, 2, 64
    ws = L.fgfrft_apply_operator_workspace_bytes(N, n, B, 0)
    for Q, X, Y, W in ((0x100008, 0x200000, 0x300000, 0x400000), (0x100000, 0x200004, 0x300000, 0x400000),
                       (0x100000, 0x200000, 0x300004, 0x400000), (0x100000, 0x200000, 0x300000, 0x400040)):
        rc = L.fgfrft_apply_operator(P(Q), N, n, 0, P(X), 0, 0, B, P(Y), 0, P(W), ws, None)
        assert rc == -1 and b"aligned" in L.fgfrft_last_error(), (Q, X, Y, W)
    wsx = L.fgfrft_gfrft_exact_workspace_bytes(N)
    for V, Vh, th, out, W in ((0x100004, 0x200000, 0x300000, 0x400000, 0x500000),
                              (0x100000, 0x200000, 0x300000, 0x400000, 0x500010)):
        rc = L.fgfrft_gfrft_exact(P(V), P(Vh), P(th), N, 0.5, P(out), P(W), wsx, None)
        assert rc == -1 and b"aligned" in L.fgfrft_last_error(), (V, W)


def test_header_is_plain_c_and_the_library_links_from_c(L, tmp_path):
    """The boundary is usable from C: the header compiles as C99 with pedantic warnings as errors,
    and a C program linked against the library queries plan sizes (host-only calls)."""
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "use_abi.c"
    src.write_text(
        "#include <stdio.h>\n#include \"fgfrft.h\"\n"
        "int main(void) {\n"
        "  size_t p = 0, s = 0;\n"
        "  fgfrft_status rc = fgfrft_plan_bytes(64, 8, FGFRFT_IN_F64, FGFRFT_STACK_FP32, &p, &s);\n"
        "  printf(\"%d %zu %s\\n\", (int)rc, p, fgfrft_strerror(FGFRFT_EALPHA));\n"
        "  return rc == FGFRFT_OK ? 0 : 1;\n}\n")
    libdir = os.path.dirname(_lib.LIB_PATH)
    exe = tmp_path / "use_abi"
    r = subprocess.run([gcc, "-std=c99", "-Wall", "-Wextra", "-pedantic", "-Werror", "-I", os.path.join(ROOT, "include"),
                        str(src), "-L", libdir, "-lfgfrft", f"-Wl,-rpath,{libdir}", "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stderr
    rc, pbytes, msg = r.stdout.split(" ", 2)
    assert rc == "0" and int(pbytes) >= 2 * 8 * 64 * 64 * 4 + 64 * 64 * 4
    assert msg.startswith("order out of range")


def test_binding_signatures_match_the_header_prototypes():
    """Every prototype's parameter count equals the binding's ctypes argtypes, and pointer
    parameters are passed as pointers: a shifted argument would hand a kernel a wrong address."""
    import ctypes
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    protos = dict((name, params) for name, params in
                  re.findall(r"FGFRFT_API\s+[\w\s\*]+?\b(fgfrft_\w+)\s*\(([^)]*)\)\s*;", text))
    assert set(protos) == set(_lib.SIGNATURES)
    for name, params in protos.items():
        ps = [p.strip() for p in params.split(",")] if params.strip() not in ("", "void") else []
        _, argtypes = _lib.SIGNATURES[name]
        assert len(ps) == len(argtypes), name
        scalar = {"int": ctypes.c_int, "double": ctypes.c_double, "size_t": ctypes.c_size_t,
                  "fgfrft_plan_t": ctypes.c_void_p}
        for p, t in zip(ps, argtypes):
            if "*" in p:
                assert t is ctypes.c_void_p or t is ctypes.c_char_p or issubclass(t, ctypes._Pointer), (name, p, t)
            else:   # a size_t passed as a 32-bit int would leave the register's upper half undefined
                ctype = p.replace("const ", "").split()[0]
                assert scalar[ctype] is t, (name, p, t)


def test_binding_constants_match_the_header_enums():
    """Status codes, stack types and forms the binding passes as integers are the header's values."""
    text = open(HEADER).read()
    enum = {name: int(val) for name, val in re.findall(r"\b(FGFRFT_[A-Z0-9_]+)\s*=\s*(-?\d+)", text)}
    for code, name in _lib.STATUS.items():
        assert enum[name] == code, name
    from paper_2602_20870_amd import ops
    assert ops.STACK_TYPES == {"fp32": enum["FGFRFT_STACK_FP32"], "bf16x2": enum["FGFRFT_STACK_BF16X2"],
                               "fp16x2": enum["FGFRFT_STACK_FP16X2"]}
    assert ops.FORMS == {"split": enum["FGFRFT_FORM_SPLIT"], "standard": enum["FGFRFT_FORM_STANDARD"]}
    assert (enum["FGFRFT_IN_C128"], enum["FGFRFT_IN_F64"]) == (0, 1)   # the intype ops.Plan passes


def test_strerror_names(L):
    for code in range(0, -8, -1):
        assert L.fgfrft_strerror(code)
    assert L.fgfrft_strerror(-3).startswith(b"order out of range")
