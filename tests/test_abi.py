"""The C ABI on the CPU: the library loads, exports every entry point that
include/*.h declares (mimo_cg.h, mimo_serve.h), and rejects invalid
arguments synchronously (before any HIP call).  No kernel runs here."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

from paper_1404_0424_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mimo_cg.h")
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))


def _declared():
    names = set()
    for h in HEADERS:
        src = re.sub(r"/\*.*?\*/", "", open(h).read(), flags=re.S)
        names |= set(re.findall(r"\b(mimo_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = _declared()
    for need in ("mimo_gram_mf", "mimo_detect_cg", "mimo_precode_cg", "mimo_convert",
                 "mimo_workspace_bytes", "mimo_status_string", "mimo_last_error"):
        assert need in names


def test_library_exports_every_declared_symbol():
    lib = L.lib()
    for name in _declared():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True,
                         text=True).stdout
    exported = set(re.findall(r"\bT (mimo_\w+)", out))
    assert set(_declared()) <= exported


def test_headers_compile_as_c_and_link(tmp_path):
    """include/*.h are plain C: a C11 translation unit that includes them and
    calls every compute entry point (returning mimo_status) compiles without
    warnings and links against the library."""
    src = tmp_path / "use.c"
    src.write_text(
        '#include "mimo_cg.h"\n#include "mimo_serve.h"\n'
        "int main(void) {\n"
        "  mimo_shape s = {32, 8, 1, 3, 0};\n"
        "  mimo_status st = mimo_detect_cg(&s, 0, 0, MIMO_C32, 1.f, 1.f, 4, MIMO_SINR_APPROX,\n"
        "                                  MIMO_SCALAR_F32, 0, 0, 0, 0, 0, 0, 0);\n"
        "  st = mimo_precode_cg(&s, 0, 0, MIMO_C32, 0.f, 0, MIMO_SCALAR_F32, 0, 0, 0, 0, 0);\n"
        "  st = mimo_gram_mf(&s, 0, 0, MIMO_C32, 0.f, 0, 0, 0);\n"
        "  return mimo_status_string(st) == 0;\n"
        "}\n")
    exe = tmp_path / "use"
    r = subprocess.run(["gcc", "-std=c11", "-Wall", "-Wextra", "-Werror", "-I",
                        os.path.join(ROOT, "include"), str(src), L.LIB_PATH, "-o", str(exe)],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr


def test_header_constants_match_binding():
    src = open(HEADER).read()
    assert re.search(rf"#define MIMO_MAX_USERS {L.MIMO_MAX_USERS}\b", src)
    assert re.search(rf"#define MIMO_MAX_USERS_COMMON {L.MIMO_MAX_USERS_COMMON}\b", src)
    assert f"#define MIMO_MAX_ANTENNAS {L.MIMO_MAX_ANTENNAS}" in src
    assert f"#define MIMO_MAX_BATCH {L.MIMO_MAX_BATCH}" in src
    m = re.search(r"#define MIMO_MAX_SPAN_BYTES (\d+)LL", src)
    assert m and int(m.group(1)) == L.MIMO_MAX_SPAN_BYTES
    for name in ("MIMO_C32", "MIMO_C16", "MIMO_CBF16", "MIMO_SINR_APPROX", "MIMO_SINR_EXACT",
                 "MIMO_SCALAR_F32", "MIMO_SCALAR_F64", "MIMO_OK", "MIMO_EINVAL",
                 "MIMO_EUNSUPPORTED", "MIMO_EWORKSPACE", "MIMO_EHIP"):
        m = re.search(rf"\b{name}\s*=\s*(-?\d+)", src)
        assert m and int(m.group(1)) == getattr(L, name), name


# fake, aligned, never-dereferenced device addresses for validation tests
P = 0x100000
P2 = 0x200000


def _detect(shape, **kw):
    a = dict(H=P, Y=P, dt=0, n0=0.5, es=1.0, m=4, mode=0, prec=0, llr=P2, xhat=None, mu=None,
             sinr=None)
    a.update(kw)
    return L.lib().mimo_detect_cg(shape, a["H"], a["Y"], a["dt"], a["n0"], a["es"], a["m"],
                                  a["mode"], a["prec"], a["llr"], a["xhat"], a["mu"], a["sinr"],
                                  None, 0, None)


@pytest.mark.parametrize("shape,kw,status", [
    ((32, 8, 1, 3, 4), dict(n0=0.0), L.MIMO_EINVAL),
    ((32, 8, 1, 3, 4), dict(n0=float("nan")), L.MIMO_EINVAL),
    ((32, 8, 1, 3, 4), dict(es=-1.0), L.MIMO_EINVAL),
    ((32, 8, 1, 3, 4), dict(m=3), L.MIMO_EUNSUPPORTED),
    ((32, 8, 1, 3, 4), dict(m=10), L.MIMO_EUNSUPPORTED),
    ((32, 8, 1, 3, 4), dict(mode=2), L.MIMO_EINVAL),
    ((32, 8, 1, 3, 4), dict(prec=7), L.MIMO_EINVAL),
    ((32, 8, 1, 3, 4), dict(dt=5), L.MIMO_EINVAL),
    ((30, 8, 1, 3, 4), dict(dt=1), L.MIMO_EINVAL),          # 16-bit needs B % 8 == 0
    ((32, 8, 1, 3, 4), dict(H=None), L.MIMO_EINVAL),
    ((32, 8, 1, 3, 4), dict(Y=None), L.MIMO_EINVAL),
    ((32, 8, 1, 3, 4), dict(llr=None), L.MIMO_EINVAL),
    ((32, 8, 1, 3, 4), dict(H=P + 8), L.MIMO_EINVAL),        # misaligned
    ((32, 8, 1, 0, 4), {}, L.MIMO_EINVAL),                   # K < 1
    ((32, 8, 0, 3, 4), {}, L.MIMO_EINVAL),                   # S < 1
    ((4, 8, 1, 3, 4), {}, L.MIMO_EINVAL),                    # B < U
    ((32, 0, 1, 3, 4), {}, L.MIMO_EINVAL),                   # U < 1
    ((128, 65, 1, 3, 4), {}, L.MIMO_EUNSUPPORTED),           # U > MIMO_MAX_USERS
    ((64, 33, 1, 3, 4), dict(mode=1), L.MIMO_EUNSUPPORTED),  # exact SINR, U > 32
    ((64, 33, 1, 3, 4), dict(dt=1), L.MIMO_EUNSUPPORTED),    # 16-bit storage, U > 32
    ((64, 40, 1, 3, 4), dict(dt=2), L.MIMO_EUNSUPPORTED),
    ((32, 8, 1, 3, -1), {}, L.MIMO_EINVAL),                  # n_sc < 0
])
def test_detect_rejects_invalid_arguments(shape, kw, status):
    st = _detect(L.shape(*shape), **kw)
    assert st == status
    assert L.lib().mimo_last_error()


def _max_s(B, U):
    """Largest S whose per-subcarrier arrays stay below MIMO_MAX_SPAN_BYTES."""
    return (L.MIMO_MAX_SPAN_BYTES - 1) // (8 * max(B, 4 * U))


@pytest.mark.parametrize("B,U", [(4096, 32), (128, 16), (32, 8), (64, 32)])
def test_rhs_count_bounded_by_32bit_offsets(B, U):
    """Per-subcarrier arrays are addressed with 32-bit byte offsets (2^31 marks
    a masked lane): an S whose Y / Q (8 B S bytes) or LLR (32 U S bytes) range
    reaches 2^31 is rejected before anything is enqueued, on every entry point
    that takes a shape; the largest S below the bound passes validation (with
    n_sc = 0, so nothing runs)."""
    lib = L.lib()
    s_ok, s_bad = _max_s(B, U), _max_s(B, U) + 1
    assert 8 * max(B, 4 * U) * s_bad >= L.MIMO_MAX_SPAN_BYTES
    for S, n_sc, want in ((s_bad, 4, L.MIMO_EUNSUPPORTED), (s_bad, 0, L.MIMO_EUNSUPPORTED),
                          (s_ok, 0, L.MIMO_OK)):
        sh = L.shape(B, U, S, 3, n_sc)
        assert _detect(sh, m=8) == want
        assert lib.mimo_precode_cg(sh, P, P, 0, 0.1, 0, 0, P2, None, None, 0, None) == want
        assert lib.mimo_gram_mf(sh, P, P, 0, 0.5, P2, P2, None) == want
        assert lib.mimo_detect_cholesky(sh, P, P, 0, 0.5, 1.0, 4, P2, None, None, None,
                                        None) == want
        assert lib.mimo_precode_cgls(sh, P, P, 0, 0.1, 0, 0, P2, None, None) == want
        if want != L.MIMO_OK:
            assert b"too large" in lib.mimo_last_error()
    fr = (L.MimoFrame * 1)()
    fr[0] = L.MimoFrame(4, B, U, s_bad, 3, P, P, P2, None, 0.5, 1.0, 0.0, 0)
    assert lib.mimo_detect_cg_batch(ctypes.addressof(fr), 1, 0, 4, 0,
                                    None) == L.MIMO_EUNSUPPORTED


def test_users_beyond_32_validation():
    """33 <= U <= MIMO_MAX_USERS passes validation on the CG detection
    (approximate SINR), precoding, slot and Gram calls with complex64 storage
    (n_sc = 0 here, so nothing runs) and is rejected with MIMO_EUNSUPPORTED by
    every call that is not built for it."""
    lib = L.lib()
    for U in (33, 48, L.MIMO_MAX_USERS):
        empty = L.shape(128, U, 14, 4, 0)
        assert _detect(empty) == L.MIMO_OK
        assert _detect(empty, prec=1, m=8) == L.MIMO_OK
        assert lib.mimo_precode_cg(empty, P, P, 0, 0.1, 1, 0, P2, None, None, 0,
                                   None) == L.MIMO_OK
        s = L.shape(128, U, 14, 4, 4)
        assert lib.mimo_precode_cg(s, P, P, 1, 0.1, 1, 0, P2, None, None, 0,
                                   None) == L.MIMO_EUNSUPPORTED
        assert lib.mimo_gram_mf(empty, P, P, 0, 0.5, P2, P2, None) == L.MIMO_OK
        assert lib.mimo_gram_mf(s, P, P, 2, 0.5, P2, P2, None) == L.MIMO_EUNSUPPORTED
        assert lib.mimo_detect_cholesky(s, P, P, 0, 0.5, 1.0, 4, P2, None, None, None,
                                        None) == L.MIMO_EUNSUPPORTED
        assert lib.mimo_detect_neumann(s, P, P, 0, 0.5, 1.0, 4, P2, None, None, None,
                                       None) == L.MIMO_EUNSUPPORTED
        assert lib.mimo_precode_cholesky(s, P, P, 0, 0.1, 0, P2, None,
                                         None) == L.MIMO_EUNSUPPORTED
        assert lib.mimo_detect_cgls(s, P, P, 0, 0.5, 1.0, 4, 0, P2, None, None, None,
                                    None) == L.MIMO_EUNSUPPORTED
        assert lib.mimo_precode_cgls(s, P, P, 0, 0.1, 0, 0, P2, None,
                                     None) == L.MIMO_EUNSUPPORTED
        fr = (L.MimoFrame * 1)()
        fr[0] = L.MimoFrame(4, 128, U, 14, 4, P, P, P2, None, 0.5, 1.0, 0.1, 1)
        assert lib.mimo_detect_cg_batch(ctypes.addressof(fr), 1, 0, 4, 0,
                                        None) == L.MIMO_EUNSUPPORTED
        assert lib.mimo_precode_cg_batch(ctypes.addressof(fr), 1, 0, 0,
                                         None) == L.MIMO_EUNSUPPORTED
        assert b"U=" in lib.mimo_last_error()


def test_cached_gram_validation():
    """mimo_detect_cg_gram / mimo_precode_cg_gram validate like the direct
    calls and require an aligned G; U beyond 32 is not built for them."""
    lib = L.lib()
    s = L.shape(32, 8, 2, 3, 4)
    det = lambda sh, G, **kw: lib.mimo_detect_cg_gram(sh, G, P, P, 0, kw.get("n0", 0.5), 1.0,
                                                       kw.get("m", 4), 0, P2, None, None, None,
                                                       None)
    pre = lambda sh, G, **kw: lib.mimo_precode_cg_gram(sh, G, P, P, 0, kw.get("beta", 0.1), 1, 0,
                                                        P2, None, None)
    for fn in (det, pre):
        assert fn(s, None) == L.MIMO_EINVAL
        assert fn(s, P + 8) == L.MIMO_EINVAL
        assert fn(L.shape(32, 8, 2, 3, 0), P) == L.MIMO_OK
        assert fn(L.shape(128, 33, 2, 3, 4), P) == L.MIMO_EUNSUPPORTED
        assert fn(L.shape(4, 8, 2, 3, 4), P) == L.MIMO_EINVAL             # B < U
    assert det(s, P, n0=0.0) == L.MIMO_EINVAL
    assert det(s, P, m=5) == L.MIMO_EUNSUPPORTED
    assert pre(s, P, beta=-1.0) == L.MIMO_EINVAL
    fr = (L.MimoFrame * 1)()
    fr[0] = L.MimoFrame(4, 32, 8, 2, 3, P, P, P2, None, 0.5, 1.0, 0.0, 0, P + 4)
    assert lib.mimo_detect_cg_batch(ctypes.addressof(fr), 1, 0, 4, 0, None) == L.MIMO_EINVAL
    assert b"gram" in lib.mimo_last_error()


def test_zero_subcarriers_is_a_noop():
    assert _detect(L.shape(32, 8, 14, 3, 0)) == L.MIMO_OK


def test_precode_gram_convert_validation():
    lib = L.lib()
    s = L.shape(32, 8, 2, 3, 4)
    assert lib.mimo_precode_cg(s, P, P, 0, -0.1, 0, 0, P2, None, None, 0, None) == L.MIMO_EINVAL
    assert lib.mimo_precode_cg(s, P, None, 0, 0.1, 0, 0, P2, None, None, 0, None) == L.MIMO_EINVAL
    assert lib.mimo_precode_cg(s, P, P, 0, 0.1, 0, 0, None, None, None, 0, None) == L.MIMO_EINVAL
    assert lib.mimo_precode_cg(L.shape(32, 8, 2, 3, 0), P, P, 0, 0.0, 1, 1, P2, None, None, 0,
                               None) == L.MIMO_OK
    assert lib.mimo_gram_mf(s, P, None, 0, -1.0, P2, None, None) == L.MIMO_EINVAL
    assert lib.mimo_gram_mf(s, P, None, 0, 0.5, P2, P2, None) == L.MIMO_EINVAL   # b without Y
    assert lib.mimo_gram_mf(L.shape(32, 8, 2, 3, 0), P, P, 0, 0.5, P2, P2, None) == L.MIMO_OK
    assert lib.mimo_convert(P, P2, 0, 4, 32, 8, None) == L.MIMO_EINVAL          # dst not 16-bit
    assert lib.mimo_convert(P, P2, 1, 4, 30, 8, None) == L.MIMO_EINVAL          # R % 8
    assert lib.mimo_convert(P, P2, 2, 0, 32, 8, None) == L.MIMO_OK
    assert lib.mimo_workspace_bytes(s, 1, 0) == 0


def test_comparison_methods_validation():
    lib = L.lib()
    s = L.shape(32, 8, 2, 3, 4)
    for fn in (lib.mimo_detect_cholesky, lib.mimo_detect_neumann):
        assert fn(s, P, P, 0, 0.0, 1.0, 4, P2, None, None, None, None) == L.MIMO_EINVAL   # n0
        assert fn(s, P, P, 0, 0.5, 1.0, 5, P2, None, None, None, None) == L.MIMO_EUNSUPPORTED
        assert fn(s, P, None, 0, 0.5, 1.0, 4, P2, None, None, None, None) == L.MIMO_EINVAL
        assert fn(s, P, P, 0, 0.5, 1.0, 4, P2 + 4, None, None, None, None) == L.MIMO_EINVAL
        assert fn(L.shape(32, 8, 2, 3, 0), P, P, 0, 0.5, 1.0, 4, P2, None, None, None,
                  None) == L.MIMO_OK
    # Neumann needs K >= 1 terms; the Cholesky detector ignores K
    k0 = L.shape(32, 8, 2, 0, 0)
    assert lib.mimo_detect_neumann(k0, P, P, 0, 0.5, 1.0, 4, P2, None, None, None,
                                   None) == L.MIMO_EINVAL
    assert lib.mimo_detect_cholesky(k0, P, P, 0, 0.5, 1.0, 4, P2, None, None, None,
                                    None) == L.MIMO_OK
    for fn in (lib.mimo_precode_cholesky, lib.mimo_precode_neumann):
        assert fn(s, P, P, 0, -1.0, 0, P2, None, None) == L.MIMO_EINVAL               # beta
        assert fn(s, P, P, 0, 0.1, 0, None, None, None) == L.MIMO_EINVAL              # Q
        assert fn(L.shape(30, 8, 2, 3, 4), P, P, 1, 0.1, 0, P2, None, None) == L.MIMO_EINVAL
        assert fn(L.shape(32, 8, 2, 3, 0), P, P, 0, 0.0, 1, P2, None, None) == L.MIMO_OK
    assert lib.mimo_precode_neumann(k0, P, P, 0, 0.1, 0, P2, None, None) == L.MIMO_EINVAL


def _slot(ul, dl, **kw):
    a = dict(H=P, Y=P, T=P, dt=0, n0=0.5, es=1.0, m=4, beta=0.5, norm=1, prec=0, llr=P2,
             xhat=None, mu=None, sinr=None, Q=P2, qnorm=None)
    a.update(kw)
    return L.lib().mimo_detect_precode_cg(ul, dl, a["H"], a["Y"], a["T"], a["dt"], a["n0"],
                                          a["es"], a["m"], a["beta"], a["norm"], a["prec"],
                                          a["llr"], a["xhat"], a["mu"], a["sinr"], a["Q"],
                                          a["qnorm"], None)


def test_slot_validation_without_a_gpu():
    """mimo_detect_precode_cg: both shapes must describe one channel (B, U,
    n_sc); S and K may differ; every argument is checked before anything is
    enqueued, and n_sc = 0 is a no-op."""
    ul, dl = L.shape(32, 8, 14, 3, 4), L.shape(32, 8, 5, 6, 4)
    for kw, want in ((dict(n0=0.0), L.MIMO_EINVAL), (dict(es=-1.0), L.MIMO_EINVAL),
                     (dict(beta=-0.1), L.MIMO_EINVAL), (dict(beta=float("inf")), L.MIMO_EINVAL),
                     (dict(m=5), L.MIMO_EUNSUPPORTED), (dict(prec=3), L.MIMO_EINVAL),
                     (dict(dt=4), L.MIMO_EINVAL), (dict(H=None), L.MIMO_EINVAL),
                     (dict(Y=None), L.MIMO_EINVAL), (dict(T=None), L.MIMO_EINVAL),
                     (dict(llr=None), L.MIMO_EINVAL), (dict(Q=None), L.MIMO_EINVAL),
                     (dict(qnorm=P2 + 4), L.MIMO_EINVAL), (dict(xhat=P + 8), L.MIMO_EINVAL)):
        assert _slot(ul, dl, **kw) == want, kw
        assert L.lib().mimo_last_error()
    for other in (L.shape(64, 8, 5, 6, 4), L.shape(32, 4, 5, 6, 4), L.shape(32, 8, 5, 6, 5)):
        assert _slot(ul, other) == L.MIMO_EINVAL
        assert b"share the channel" in L.lib().mimo_last_error()
    assert _slot(ul, L.shape(32, 8, 5, 0, 4)) == L.MIMO_EINVAL             # K_dl < 1
    assert _slot(L.shape(32, 8, 0, 3, 4), dl) == L.MIMO_EINVAL             # S_ul < 1
    assert _slot(L.shape(128, 65, 2, 3, 4), L.shape(128, 65, 2, 3, 4)) == L.MIMO_EUNSUPPORTED
    assert _slot(L.shape(64, 33, 2, 3, 4), L.shape(64, 33, 2, 3, 4), dt=1) == L.MIMO_EUNSUPPORTED
    assert _slot(L.shape(64, 64, 2, 3, 0), L.shape(64, 64, 5, 2, 0)) == L.MIMO_OK
    assert _slot(L.shape(32, 8, 14, 3, 0), L.shape(32, 8, 5, 6, 0)) == L.MIMO_OK
    assert L.lib().mimo_tune_variant_count(L.MIMO_OP_SLOT) == 3
    assert L.lib().mimo_tune_variant_name(L.MIMO_OP_SLOT, 1) == b"fused"


def test_status_strings():
    lib = L.lib()
    for st in (0, -1, -2, -3, -4):
        assert lib.mimo_status_string(st)
    assert b"unknown" in lib.mimo_status_string(99)
    assert lib.mimo_version().startswith(b"mimo_cg")


def test_schedule_table_validation_and_roundtrip():
    import ctypes as C
    lib = L.lib()
    assert lib.mimo_tune_variant_count(L.MIMO_OP_DETECT) >= 1
    names = [lib.mimo_tune_variant_name(L.MIMO_OP_DETECT, v)
             for v in range(lib.mimo_tune_variant_count(L.MIMO_OP_DETECT))]
    assert all(names) and names[0] == b"generic"
    assert lib.mimo_tune_variant_name(L.MIMO_OP_DETECT, 99) is None
    assert lib.mimo_tune_set(7, 0, 0, 0, 0) == L.MIMO_EINVAL
    assert lib.mimo_tune_set(L.MIMO_OP_DETECT, 2, 0, 0, 0) == L.MIMO_EINVAL
    assert lib.mimo_tune_set(L.MIMO_OP_DETECT, 0, 3, 0, 0) == L.MIMO_EINVAL
    assert lib.mimo_tune_set(L.MIMO_OP_DETECT, 0, 0, 99, 0) == L.MIMO_EINVAL
    assert lib.mimo_tune_set(L.MIMO_OP_DETECT, 0, 0, 0, 65) == L.MIMO_EINVAL
    v0, b0 = C.c_int(), C.c_int()
    assert lib.mimo_tune_get(L.MIMO_OP_DETECT, 1, 2, C.byref(v0), C.byref(b0)) == L.MIMO_OK
    assert lib.mimo_tune_set(L.MIMO_OP_DETECT, 1, 2, 1, 3) == L.MIMO_OK
    v, b = C.c_int(), C.c_int()
    assert lib.mimo_tune_get(L.MIMO_OP_DETECT, 1, 2, C.byref(v), C.byref(b)) == L.MIMO_OK
    assert (v.value, b.value) == (1, 3)
    assert lib.mimo_tune_set(L.MIMO_OP_DETECT, 1, 2, v0.value, b0.value) == L.MIMO_OK


def test_autotune_table_save_load(tmp_path):
    from paper_1404_0424_amd import autotune
    entries = [{"op": "detect", "user_class": 0, "dtype": 1,
                "best": {"variant": 2, "blocks_per_cu": 4, "seconds": 1e-4}}]
    p = tmp_path / "t.json"
    before = autotune.get_schedule("detect", 8, 1)
    autotune.save(entries, str(p))
    assert autotune.load(str(p)) == 1
    assert autotune.get_schedule("detect", 8, 1) == (2, 4)
    autotune.set_schedule("detect", 8, 1, *before)


def test_batch_validation():
    lib = L.lib()
    fr = (L.MimoFrame * 2)()
    fr[0] = L.MimoFrame(4, 32, 8, 2, 3, P, P, P2, None, 0.5, 1.0, 0.0, 0)
    fr[1] = L.MimoFrame(4, 32, 8, 2, 3, P, P, P2, None, -0.5, 1.0, 0.0, 0)   # bad n0
    st = lib.mimo_detect_cg_batch(ctypes.addressof(fr), 2, 0, 4, 0, None)
    assert st == L.MIMO_EINVAL and b"frame 1" in lib.mimo_last_error()
    fr[1] = L.MimoFrame(4, 64, 40, 2, 3, P, P, P2, None, 0.5, 1.0, 0.0, 0)   # U too large
    assert lib.mimo_detect_cg_batch(ctypes.addressof(fr), 2, 0, 4, 0, None) == L.MIMO_EUNSUPPORTED
    assert lib.mimo_detect_cg_batch(ctypes.addressof(fr), 33, 0, 4, 0, None) == L.MIMO_EINVAL
    assert lib.mimo_detect_cg_batch(None, 1, 0, 4, 0, None) == L.MIMO_EINVAL
    assert lib.mimo_detect_cg_batch(ctypes.addressof(fr), 1, 0, 5, 0, None) == L.MIMO_EUNSUPPORTED
    fr[0] = L.MimoFrame(0, 32, 8, 2, 3, P, P, P2, None, 0.5, 1.0, 0.0, 0)    # empty frame
    assert lib.mimo_detect_cg_batch(ctypes.addressof(fr), 1, 0, 4, 0, None) == L.MIMO_OK
    assert lib.mimo_detect_cg_batch(ctypes.addressof(fr), 0, 0, 4, 0, None) == L.MIMO_OK
    fr[0] = L.MimoFrame(4, 32, 8, 2, 3, P, P, P2, None, 0.0, 0.0, -1.0, 1)   # bad beta
    assert lib.mimo_precode_cg_batch(ctypes.addressof(fr), 1, 0, 0, None) == L.MIMO_EINVAL


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    """Without the built library every entry point raises; nothing falls back
    to a CPU computation."""
    from paper_1404_0424_amd import api
    monkeypatch.setattr(L, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(L, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        api.workspace_bytes(128, 16, 14, 4, 1200)
    with pytest.raises(RuntimeError, match="missing"):
        L.lib()


def test_product_package_does_not_import_the_oracle():
    """The oracle is test infrastructure: no module of the package imports it,
    and importing the package loads no oracle module."""
    pkg = os.path.join(ROOT, "paper_1404_0424_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                src = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle\b", src, re.M), f
    code = ("import sys, paper_1404_0424_amd, paper_1404_0424_amd.api, "
            "paper_1404_0424_amd.serving, paper_1404_0424_amd.autotune; "
            "print(any(m == 'oracle' or m.startswith('oracle.') for m in sys.modules))")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                         timeout=120)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip() == "False"


def test_server_validation_without_a_gpu():
    """The native server's entry points reject bad configurations and NULL
    handles before any HIP call."""
    import ctypes
    lib = L.lib()
    out = ctypes.c_void_p()
    for cfg in [L.MimoServerConfig(0, 4, 32, 128, 0, 1), L.MimoServerConfig(1 << 20, 0, 32, 128, 0, 1),
                L.MimoServerConfig(1 << 20, L.MIMO_SERVE_MAX_SLOTS + 1, 32, 128, 0, 1),
                L.MimoServerConfig(1 << 20, 4, 0, 128, 0, 1),
                L.MimoServerConfig(1 << 20, 4, L.MIMO_MAX_BATCH + 1, 128, 0, 1),
                L.MimoServerConfig(1 << 20, 4, 32, 0, 0, 1)]:
        assert lib.mimo_server_create(ctypes.byref(cfg), 0, ctypes.byref(out)) == L.MIMO_EINVAL
        assert lib.mimo_last_error()
    assert lib.mimo_server_create(None, 0, ctypes.byref(out)) == L.MIMO_EINVAL
    rid = ctypes.c_int64()
    up = L.MimoUplinkReq()
    dn = L.MimoDownlinkReq()
    assert lib.mimo_server_destroy(None) == L.MIMO_EINVAL
    assert lib.mimo_server_register_channel(None, 1, P, 0, 1, 8, 4) == L.MIMO_EINVAL
    assert lib.mimo_server_register_channel_gram(None, 1, P, P, 0, 1, 8, 4) == L.MIMO_EINVAL
    assert lib.mimo_server_unregister_channel(None, 1) == L.MIMO_EINVAL
    assert lib.mimo_server_submit_uplink(None, ctypes.byref(up), None, ctypes.byref(rid)) == L.MIMO_EINVAL
    assert lib.mimo_server_submit_downlink(None, ctypes.byref(dn), None, ctypes.byref(rid)) == L.MIMO_EINVAL
    assert lib.mimo_server_poll(None, None, 0, 0) == L.MIMO_EINVAL
    assert lib.mimo_server_release(None, 1) == L.MIMO_EINVAL
    assert lib.mimo_server_dlpack(None, 1, 0, ctypes.byref(out)) == L.MIMO_EINVAL
    assert lib.mimo_server_pause(None) == L.MIMO_EINVAL
    assert lib.mimo_server_resume(None) == L.MIMO_EINVAL
    assert lib.mimo_server_drain(None, 0) == L.MIMO_EINVAL
    st = L.MimoServerStats()
    assert lib.mimo_server_stats_get(None, 0, 0, ctypes.byref(st)) == L.MIMO_EINVAL
    assert lib.mimo_server_memory(None, None, None) == L.MIMO_EINVAL


def test_serve_header_constants_match_binding():
    src = open(os.path.join(ROOT, "include", "mimo_serve.h")).read()
    assert f"#define MIMO_SERVE_MAX_SLOTS {L.MIMO_SERVE_MAX_SLOTS}" in src
    # struct layouts the binding relies on (sizes of the C structs)
    import ctypes
    assert ctypes.sizeof(L.MimoServerConfig) == 32
    assert ctypes.sizeof(L.MimoUplinkReq) == 48
    assert ctypes.sizeof(L.MimoDownlinkReq) == 40
    assert ctypes.sizeof(L.MimoCompletion) == 96
