"""The C ABI loads, exports every declared symbol and rejects bad arguments on
the host, before any device work (runs without a GPU)."""

import ctypes as C
import os
import subprocess

import pytest

from paper_2305_13925_amd import binding as bd

L = bd.lib()
NULL = None
FAKE = C.c_void_p(0x1000)      # never dereferenced: validation fails first


def _err():
    return bd.last_error()


def test_exports_every_declared_symbol():
    declared = bd.exported_symbols()
    assert {"jacpcg_gram", "jacpcg_solve", "rzf_precoder", "rzf_precoder_plain",
            "jacpcg_session_create", "jacpcg_session_destroy"} <= set(declared)
    out = subprocess.run(["nm", "-D", "--defined-only", bd.LIB_PATH], capture_output=True, text=True).stdout
    exported = {line.split()[-1] for line in out.splitlines() if " T " in line}
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert hasattr(L, s)


def test_version_and_status_strings():
    assert L.jacpcg_version() >= 10000
    for code in (0, 1, 2, -1, -2, -3, -4, -5, -6, -7, -8, -9):
        assert bd.status_string(code) != "unknown status"
    assert bd.status_string(12345) == "unknown status"


def test_session_create_argument_errors():
    h = C.c_void_p()
    assert L.jacpcg_session_create(0, 0, None, None) == bd.E_INVALID_ARG
    assert L.jacpcg_session_create(-1, 0, None, C.byref(h)) == bd.E_INVALID_ARG
    assert "device" in _err()


def _gram(**kw):
    a = dict(s=NULL, stream=NULL, batch=2, M=64, K=16, H=FAKE, ldh=64, sh=64 * 16, xi=1.0, prec=0,
             A=FAKE, lda=16, sa=256, diag=NULL)
    a.update(kw)
    return L.jacpcg_gram(a["s"], a["stream"], a["batch"], a["M"], a["K"], a["H"], a["ldh"], a["sh"], a["xi"],
                         a["prec"], a["A"], a["lda"], a["sa"], a["diag"])


@pytest.mark.parametrize("kw,word", [
    (dict(K=0), "K"), (dict(K=257), "K"), (dict(M=0), "M"), (dict(batch=-1), "batch"),
    (dict(xi=-1.0), "xi"), (dict(xi=float("nan")), "xi"), (dict(ldh=63), "ldh"),
    (dict(sh=64 * 16 - 1), "stride_h"), (dict(H=NULL), "H"), (dict(A=NULL), "A"), (dict(lda=15), "lda"),
])
def test_gram_validation(kw, word):
    assert _gram(**kw) == bd.E_INVALID_ARG
    assert word in _err()


def test_gram_unsupported_precision_and_null_session():
    assert _gram(prec=7) == bd.E_UNSUPPORTED
    assert _gram() == bd.E_INVALID_ARG
    assert "session" in _err()
    assert _gram(batch=0, s=NULL) == bd.E_INVALID_ARG   # valid sizes, still needs a session


def _solve(**kw):
    a = dict(s=NULL, batch=1, K=8, n=8, A=FAKE, lda=8, sa=64, B=NULL, ldb=8, sb=64, X=FAKE, ldx=8, sx=64,
             tol=0.0, it=4, flags=0)
    a.update(kw)
    return L.jacpcg_solve(a["s"], NULL, a["batch"], a["K"], a["n"], a["A"], a["lda"], a["sa"], a["B"], a["ldb"],
                          a["sb"], a["X"], a["ldx"], a["sx"], a["tol"], a["it"], a["flags"], NULL, NULL, NULL)


@pytest.mark.parametrize("kw,word", [
    (dict(n=5), "nrhs"), (dict(n=0), "nrhs"), (dict(n=300, B=FAKE), "nrhs"), (dict(tol=-1e-3), "tol"),
    (dict(it=-1), "max_iter"), (dict(flags=9), "flags"), (dict(lda=7), "lda"), (dict(ldx=3), "ldx"),
    (dict(B=FAKE, ldb=2), "ldb"), (dict(A=NULL), "A"), (dict(X=NULL), "X"), (dict(K=0), "K"),
    (dict(batch=2, sx=10), "stride_x"),
])
def test_solve_validation(kw, word):
    assert _solve(**kw) == bd.E_INVALID_ARG
    assert word in _err()


def _rzf(**kw):
    a = dict(batch=1, M=32, K=4, H=FAKE, ldh=32, sh=128, xi=0.5, power=1.0, tol=0.0, it=4, prec=0, flags=0,
             rtol=1e-10, W=FAKE, ldw=32, sw=128)
    a.update(kw)
    return L.rzf_precoder(NULL, NULL, a["batch"], a["M"], a["K"], a["H"], a["ldh"], a["sh"], a["xi"], a["power"],
                          a["tol"], a["it"], a["prec"], a["flags"], a["rtol"], a["W"], a["ldw"], a["sw"], NULL, NULL,
                          NULL)


@pytest.mark.parametrize("kw,word", [
    (dict(power=0.0), "power"), (dict(power=-2.0), "power"), (dict(W=NULL), "W"), (dict(ldw=31), "ldw"),
    (dict(tol=-1.0), "tol"), (dict(it=-3), "max_iter"), (dict(rtol=-1.0), "refine_tol"),
    (dict(xi=float("inf")), "xi"), (dict(flags=5), "flags"),
])
def test_rzf_validation(kw, word):
    assert _rzf(**kw) == bd.E_INVALID_ARG
    assert word in _err()


def test_rzf_unknown_precision():
    assert _rzf(prec=0x7) == bd.E_UNSUPPORTED
    assert _rzf(prec=0x1000) == bd.E_UNSUPPORTED


def _tx(**kw):
    a = dict(batch=2, M=32, K=4, n=3, H=FAKE, ldh=32, sh=128, S=FAKE, lds=4, ss=12, xi=0.5, power=1.0, tol=0.0,
             it=4, prec=0, flags=0, x=FAKE, ldx=32, sx=96)
    a.update(kw)
    return L.rzf_transmit(NULL, NULL, a["batch"], a["M"], a["K"], a["n"], a["H"], a["ldh"], a["sh"], a["S"],
                          a["lds"], a["ss"], a["xi"], a["power"], a["tol"], a["it"], a["prec"], a["flags"], a["x"],
                          a["ldx"], a["sx"], NULL, NULL)


@pytest.mark.parametrize("kw,word", [
    (dict(n=0), "nsym"), (dict(S=NULL), "S"), (dict(x=NULL), "x"), (dict(lds=3), "lds"),
    (dict(ss=11), "stride_s"), (dict(ldx=31), "ldx"), (dict(sx=95), "stride_x"), (dict(power=0.0), "power"),
    (dict(flags=4), "flags"), (dict(K=0), "K"),
])
def test_transmit_validation(kw, word):
    assert _tx(**kw) == bd.E_INVALID_ARG
    assert word in _err()


def test_transmit_rejects_refinement():
    assert _tx(prec=0x100) == bd.E_UNSUPPORTED
    assert _tx(prec=0x3) == bd.E_UNSUPPORTED


def _sinr(**kw):
    a = dict(batch=2, M=32, K=4, H=FAKE, ldh=32, sh=128, W=FAKE, ldw=32, sw=128, s2=0.1, sinr=FAKE, se=FAKE)
    a.update(kw)
    return L.rzf_sinr(NULL, NULL, a["batch"], a["M"], a["K"], a["H"], a["ldh"], a["sh"], a["W"], a["ldw"], a["sw"],
                      a["s2"], a["sinr"], a["se"])


@pytest.mark.parametrize("kw,word", [
    (dict(s2=-1.0), "sigma2"), (dict(s2=float("nan")), "sigma2"), (dict(W=NULL), "W"), (dict(ldw=31), "ldw"),
    (dict(sw=127), "stride_w"), (dict(sinr=NULL, se=NULL), "NULL"), (dict(K=257), "K"), (dict(H=NULL), "H"),
])
def test_sinr_validation(kw, word):
    assert _sinr(**kw) == bd.E_INVALID_ARG
    assert word in _err()


def _blk(**kw):
    a = dict(batch=2, M1=8, Mc=4, M2=8, K1=2, K2=3, H=FAKE, ldh=20, sh=100, xi=0.5, power=1.0, tol=0.0, it=4, prec=0,
             flags=0, rtol=1e-10, G=FAKE, ldg=20, sg=100)
    a.update(kw)
    return L.rzf_block_precoder(NULL, NULL, a["batch"], a["M1"], a["Mc"], a["M2"], a["K1"], a["K2"], a["H"],
                                a["ldh"], a["sh"], a["xi"], a["power"], a["tol"], a["it"], a["prec"], a["flags"],
                                a["rtol"], a["G"], a["ldg"], a["sg"], NULL)


@pytest.mark.parametrize("kw,word", [
    (dict(M1=-1), "subarray"), (dict(K2=-1), "group"), (dict(ldg=19), "ldg"), (dict(sg=99), "stride_g"),
    (dict(G=NULL), "G"), (dict(ldh=19), "ldh"), (dict(K1=200, K2=100, sh=6000, sg=6000), "K"),
    (dict(M1=0, Mc=0, M2=0), "M"), (dict(power=-1.0), "power"),
])
def test_block_validation(kw, word):
    assert _blk(**kw) == bd.E_INVALID_ARG
    assert word in _err()


def test_plain_validation():
    rc = L.rzf_precoder_plain(NULL, NULL, 1, 32, 300, FAKE, 32, 0, 0.5, 1.0, 0.0, 4, 0, FAKE, 32, 0, NULL, NULL)
    assert rc == bd.E_INVALID_ARG and "K" in _err()


def test_binding_fails_loudly_without_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(bd.JacpcgError) as ei:
        bd.Session(0)
    assert ei.value.code == bd.E_NO_DEVICE


def test_header_compiles_as_plain_c_and_structs_match_the_binding(tmp_path):
    # The public header needs no HIP header, and the ctypes mirrors of its
    # structs have the C layout (size and every field offset), as compiled by gcc.
    import ctypes as C
    import shutil
    import subprocess
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    structs = {"jacpcg_request": bd.JacpcgRequest, "jacpcg_result": bd.JacpcgResult, "jacpcg_stats": bd.JacpcgStats}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "jacpcg.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    subprocess.run([gcc, "-std=c99", "-Wall", "-Werror", "-I", os.path.join(root, "include"), str(src), "-o", str(exe)],
                   check=True, capture_output=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l}
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


def _noalloc(**kw):
    a = dict(s=NULL, batch=4, M=64, K=16, H=FAKE, ldh=64, sh=64 * 16, xi=1.0, power=1.0, tol=0.0, it=8, prec=0,
             flags=0, W=FAKE, ldw=64, sw=64 * 16, status=NULL)
    a.update(kw)
    return L.rzf_precoder_noalloc(a["s"], NULL, a["batch"], a["M"], a["K"], a["H"], a["ldh"], a["sh"], a["xi"],
                                  a["power"], a["tol"], a["it"], a["prec"], a["flags"], a["W"], a["ldw"], a["sw"],
                                  a["status"])


@pytest.mark.parametrize("kw,word", [
    (dict(K=0), "K"), (dict(M=0), "M"), (dict(xi=-1.0), "xi"), (dict(power=0.0), "power"), (dict(tol=-1.0), "tol"),
    (dict(it=-1), "max_iter"), (dict(ldw=63), "ldw"), (dict(W=NULL), "W"), (dict(flags=0x4), "flags"),
])
def test_noalloc_validation(kw, word):
    assert _noalloc(**kw) == bd.E_INVALID_ARG
    assert word in _err()


def test_noalloc_rejects_refinement_and_batches_beyond_its_scratch():
    assert _noalloc(prec=bd.GRAM_FP32 | bd.REFINE_FP64) == bd.E_UNSUPPORTED
    assert _noalloc(prec=5) == bd.E_UNSUPPORTED
    # 96 MiB: 1529 instances fit at K = 64, 383 at K = 128, 95 at K = 256; one more does not
    big = dict(M=1024, ldh=1024, ldw=1024)
    for K, fit in ((64, 1529), (128, 383), (256, 95)):
        st = dict(sh=1024 * K, sw=1024 * K, **big)
        assert _noalloc(batch=fit + 1, K=K, **st) == bd.E_INVALID_ARG
        assert "scratch" in _err()
        assert _noalloc(batch=fit, K=K, **st) == bd.E_INVALID_ARG
        assert "session" in _err()       # fits: only the missing session is left


def test_fp64_rounded_gram_needs_refinement():
    common = (NULL, NULL, 2, 64, 16, FAKE, 64, 64 * 16, 1.0, 1.0, 0.0, 8)
    rc = L.rzf_precoder(*common, bd.GRAM_FP64_ROUNDED, 0, 1e-10, FAKE, 64, 64 * 16, NULL, NULL, NULL)
    assert rc == bd.E_UNSUPPORTED
    # with refinement the precision is accepted: only the missing session is left
    rc = L.rzf_precoder(*common, bd.GRAM_FP64_ROUNDED | bd.REFINE_FP64, 0, 1e-10, FAKE, 64, 64 * 16, NULL, NULL,
                        NULL)
    assert rc == bd.E_INVALID_ARG and "session" in _err()


def test_phase_ranges_and_peak_probe_are_linked():
    # the library marks its phases with roctx ranges (rocprofv3 --marker-trace)
    out = subprocess.run(["nm", "-D", "--undefined-only", bd.LIB_PATH], capture_output=True, text=True).stdout
    assert "roctxRangePushA" in out and "roctxRangePop" in out
    # the matrix-core probe validates its arguments on the host
    assert L.jacpcg_mfma_peaks(NULL, NULL, NULL) == bd.E_INVALID_ARG


def test_tune_set_validates_knob_and_value():
    assert L.jacpcg_tune_set(NULL, b"gram_waves", 1024, 64, 2, 4) == bd.E_INVALID_ARG   # no session
    assert "session" in _err()
    assert L.jacpcg_tune_set(NULL, b"no_such_knob", 1024, 64, 2, 4) == bd.E_INVALID_ARG
    assert "unknown knob" in _err()
    for knob, bad in ((b"gram_waves", 3), (b"precoder_nj", 3), (b"precoder_mtiles", 3), (b"pcg_a_source", 5)):
        assert L.jacpcg_tune_set(NULL, knob, 1024, 64, 0, bad) == bd.E_INVALID_ARG
        assert "not a choice" in _err()
    v = C.c_int(7)
    assert L.jacpcg_tune_get(NULL, b"pcg_a_source", 0, 64, 0, C.byref(v)) == bd.E_INVALID_ARG
