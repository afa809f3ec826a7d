"""CPU-side checks of the GPU library: it builds, loads, exports every symbol the
header declares, its scalar modular arithmetic is exact, and the product code
never reaches the oracle."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ckks_lt.h")
PKG = os.path.join(ROOT, "paper_2605_17222_amd")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ckks_[a-z_0-9]+)\s*\(", text)))


def _lib_path():
    import paper_2605_17222_amd as H
    if not os.path.exists(H.LIB_PATH):
        from paper_2605_17222_amd import build
        build.build()
    return H.LIB_PATH


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "ckks_lt_eval" in names and "ckks_params_create" in names
    lib = ctypes.CDLL(_lib_path())
    for n in names:
        assert hasattr(lib, n), n
    import paper_2605_17222_amd as H
    assert sorted(H.EXPORTED) == names


def test_error_strings():
    import paper_2605_17222_amd as H
    _lib_path()
    for code in (H.CKKS_OK, H.CKKS_E_INVALID_ARG, H.CKKS_E_UNSUPPORTED, H.CKKS_E_WORKSPACE, H.CKKS_E_DEVICE,
                 H.CKKS_E_NOMEM):
        assert H.strerror(code)
    assert H.strerror(-99) == "unknown error"


def test_params_create_rejects_bad_input_without_gpu():
    # Validation happens before any device call.
    import paper_2605_17222_amd as H
    import workload as W
    _lib_path()
    prm = W.params_toy()
    with pytest.raises(H.CkksError) as e:
        H.ckks_params_create(prm.log_n, prm.q, prm.p, 2)   # dnum != ceil((L+1)/alpha)
    assert e.value.code == H.CKKS_E_INVALID_ARG
    with pytest.raises(H.CkksError):
        H.ckks_params_create(prm.log_n, (prm.q[0], prm.q[1], prm.q[1]), prm.p, 3)  # duplicate prime
    with pytest.raises(H.CkksError):
        H.ckks_params_create(prm.log_n, (prm.q[0], prm.q[1], prm.q[2] + 2), prm.p, 3)  # not prime
    with pytest.raises(H.CkksError):
        H.ckks_params_create(11, prm.q, prm.p, 3)  # ring below the supported range


def test_pack_rejects_bad_input_without_gpu():
    # ckks_pack and ckks_packed_poly_bytes check their arguments first.
    import ctypes
    import paper_2605_17222_amd as H
    _lib_path()
    L = H.lib()
    size = ctypes.c_size_t()
    assert L.ckks_packed_poly_bytes(None, ctypes.byref(size)) == H.CKKS_E_INVALID_ARG
    assert L.ckks_pack(None, 1, None, None, None) == H.CKKS_E_INVALID_ARG


def test_modarith_host_exact(tmp_path):
    src = os.path.join(ROOT, "tests", "native", "modarith_host_test.cpp")
    exe = str(tmp_path / "mah")
    subprocess.check_call(["hipcc", "-O2", "-std=c++17", src, "-o", exe], stderr=subprocess.DEVNULL)
    out = subprocess.run([exe], capture_output=True, text=True)
    assert out.returncode == 0, out.stdout
    assert " 0 failures" in out.stdout


def test_product_never_reaches_the_oracle():
    for dirpath, _, files in os.walk(PKG):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".hpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"\bimport\s+oracle|from\s+oracle|liboracle|ckks_oracle", text), f
    bench = open(os.path.join(ROOT, "bench.py")).read() if os.path.exists(os.path.join(ROOT, "bench.py")) else ""
    # the benchmark touches the oracle only inside its cpu_baseline leg
    for m in re.finditer(r"^(import oracle|from oracle)", bench, flags=re.M):
        pytest.fail("bench.py imports the oracle at module level")
