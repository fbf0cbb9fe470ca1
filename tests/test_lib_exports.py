"""The C interface: the built library loads without a GPU and exports every
function include/pcfgsmc.h declares; the Python binding names the same calls."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pcfgsmc.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(smc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def library():
    from paper_2112_00364_amd import build as B
    if B.sources_newer_than_lib():
        B.build()
    return ctypes.CDLL(B.LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("smc_model_register", "smc_init", "smc_step", "smc_resample", "smc_log_z", "smc_done",
                     "smc_batch_tick", "smc_resample_weights"):
        assert required in names


def test_every_declared_symbol_is_exported(library):
    missing = [n for n in declared_functions() if not hasattr(library, n)]
    assert not missing, missing


def test_binding_covers_the_boundary(library):
    from paper_2112_00364_amd import smc
    L = smc.lib()
    for n in declared_functions():
        assert getattr(L, n) is not None


def test_errors_without_device(library):
    """Argument checks run before any device call."""
    from paper_2112_00364_amd import smc
    L = smc.lib()
    out = ctypes.c_void_p()
    assert L.smc_ctx_create(0, None, None, None) == smc.ERR_INVALID
    assert L.smc_init(None, 10, 1, ctypes.byref(out)) == smc.ERR_INVALID
    assert L.smc_step(None) == smc.ERR_INVALID
    assert L.smc_ctx_destroy(None) == smc.OK
    assert L.smc_run_destroy(None) == smc.OK
    assert b"NULL" in L.smc_last_error()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2112_00364_amd import smc
    monkeypatch.setattr(smc, "_lib", None)
    monkeypatch.setattr(smc, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError):
        smc.lib()
