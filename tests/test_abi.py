"""CPU checks of the C-ABI library: it is built for gfx950, loads, and exports
every function include/secpe.h declares; the Python binding declares the same
set; without a GPU the product path refuses to run (no CPU fallback)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "secpe.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(secpe_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2502_00847_amd.build import lib_path as lp
    p = lp()
    if not os.path.exists(p):
        from paper_2502_00847_amd.build import build
        build()
    return p


def test_header_declares_the_boundary():
    names = _declared()
    for required in ("secpe_keygen", "secpe_encrypt", "secpe_eval_argmax", "secpe_eval_argmax_batch",
                     "secpe_decrypt", "secpe_ctx_create", "secpe_ntt_cts", "secpe_rotate_batch"):
        assert required in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_matches_header():
    from paper_2502_00847_amd import secpe
    assert sorted(secpe.exported_symbols()) == _declared()


def test_library_carries_gfx950_code(lib_path):
    out = subprocess.run(["/opt/rocm/bin/roc-obj-ls", lib_path], capture_output=True, text=True)
    if out.returncode != 0:
        pytest.skip("roc-obj-ls unavailable")
    assert "gfx950" in out.stdout


def test_no_cpu_fallback_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_2502_00847_amd.secpe import Context, SecpeError
    import workload as W
    with pytest.raises(SecpeError):
        Context(W.PARAMS["tiny"])


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2502_00847_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in re.findall(r"(?:import|from|include)\s+[\"<]?(oracle)", text)


def test_server_and_key_sharing_refuse_null_handles(lib_path):
    """Argument checks come before any device call, so they run here."""
    lib = ctypes.CDLL(lib_path)
    for name in ("secpe_server_launch", "secpe_server_ready"):
        fn = getattr(lib, name)
        fn.restype = ctypes.c_int
        fn.argtypes = [ctypes.c_void_p]
        assert fn(None) < 0
    fn = lib.secpe_server_collect
    fn.restype = ctypes.c_int
    n = ctypes.c_int(7)
    assert fn(None, 0, ctypes.byref(n), None, None, None, None, None) < 0
    fn = lib.secpe_keys_share
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert fn(None, None) < 0


def test_strerror_and_key_owner_arguments(lib_path):
    """Every status code has a fixed description; a key owner needs a context
    and a secret, and evaluations check both before any device work."""
    lib = ctypes.CDLL(lib_path)
    lib.secpe_strerror.restype = ctypes.c_char_p
    lib.secpe_strerror.argtypes = [ctypes.c_int]
    texts = {c: lib.secpe_strerror(c).decode() for c in (0, -1, -2, -3, -4, -5, -99)}
    assert len(set(texts.values())) == len(texts)
    assert "key owner" in texts[-3]
    fn = lib.secpe_key_owner_create
    fn.restype = ctypes.c_int
    fn.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]
    h = ctypes.c_void_p()
    assert fn(None, None, ctypes.byref(h)) < 0 and not h.value
    lib.secpe_key_owner_destroy.argtypes = [ctypes.c_void_p]
    lib.secpe_key_owner_destroy(None)
