"""The C-ABI library: it loads without a GPU, exports every entry point that
include/vc.h declares, and its host-only calls behave as documented.  No kernel is
launched here."""
import ctypes as C
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vc.h")
LIB = os.path.join(ROOT, "paper_2601_03031_amd", "lib", "libvc.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    text = re.sub(r"//[^\n]*", "", text)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(vc_[a-z_0-9]+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def exported():
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True, check=True).stdout
    return {ln.split()[-1] for ln in out.splitlines() if ln.strip()}


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libvc.so is not built: run __graft_entry__.build()")
    return C.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared()
    for n in ("vc_setup", "vc_commit", "vc_open_all", "vc_verify", "vc_proof_get", "vc_proof_len",
              "vc_params_free", "vc_commitment_free", "vc_proofs_free", "vc_strerror"):
        assert n in names, n


def test_every_declared_symbol_is_exported(lib):
    exp = exported()
    missing = [n for n in declared() if n not in exp]
    assert not missing, missing
    extra = sorted(n for n in exp if n.startswith("vc_") and n not in declared())
    assert not extra, "exported but undeclared: %s" % extra


def test_proof_len_matches_oracle(lib):
    import oracle as O
    lib.vc_proof_len.restype = C.c_uint64
    lib.vc_proof_len.argtypes = [C.c_uint32, C.c_uint32]
    for L in range(2, 21):
        K = 1 << (L // 2)
        for t in sorted({1, 2, K // 2 or 1, K}):
            assert lib.vc_proof_len(L, t) == O.proof_len(L, t), (L, t)


def test_strerror(lib):
    lib.vc_strerror.restype = C.c_char_p
    for code in (0, -1, -2, -3, -4, -5):
        s = lib.vc_strerror(code)
        assert s and len(s) >= 2


def test_invalid_arguments_are_rejected_without_a_device(lib):
    """Argument checks run before any device call."""
    lib.vc_setup.argtypes = [C.c_uint32, C.c_char_p, C.c_int, C.POINTER(C.c_void_p)]
    out = C.c_void_p()
    for bad in (0, 1, 31, 64):
        assert lib.vc_setup(bad, bytes(32), 0, C.byref(out)) == -1  # VC_EINVAL
    assert lib.vc_setup(4, None, 0, C.byref(out)) == -1
    assert lib.vc_setup(4, bytes(32), 0, None) == -1


def test_package_fails_loudly_without_library(tmp_path):
    """The binding refuses to run when the HIP library is missing: there is no CPU fallback."""
    code = ("import paper_2601_03031_amd as V, sys\n"
            "V.LIB_PATH = %r\n"
            "V._lib = None\n"
            "try:\n    V.lib()\nexcept (OSError, RuntimeError) as e:\n    print('raised', type(e).__name__)\n"
            "else:\n    print('loaded')\n") % str(tmp_path / "missing.so")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert "raised" in r.stdout, r.stdout + r.stderr


def test_bench_refuses_several_gpus():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
