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


def _null_calls(L):
    i, d, sz, vp = ctypes.c_int32(), ctypes.c_double(), ctypes.c_size_t(0), ctypes.c_void_p()
    return {
        "smc_set_workgroup": lambda: L.smc_set_workgroup(None, 128),
        "smc_set_bucketing": lambda: L.smc_set_bucketing(None, 1),
        "smc_snapshot": lambda: L.smc_snapshot(None, None, ctypes.byref(sz)),
        "smc_restore": lambda: L.smc_restore(None, None, 0),
        "smc_program_check": lambda: L.smc_program_check(None),
        "smc_resample": lambda: L.smc_resample(None),
        "smc_done": lambda: L.smc_done(None, ctypes.byref(i)),
        "smc_log_z": lambda: L.smc_log_z(None, ctypes.byref(d)),
        "smc_run_to_end": lambda: L.smc_run_to_end(None),
        "smc_reset": lambda: L.smc_reset(None, 1),
        "smc_read": lambda: L.smc_read(None, 0, None, 0),
        "smc_run_stats": lambda: L.smc_run_stats(None, None),
        "smc_profile": lambda: L.smc_profile(None, 1),
        "smc_profile_read": lambda: L.smc_profile_read(None, None),
        "smc_model_register": lambda: L.smc_model_register(None, None, ctypes.byref(vp)),
        "smc_batch_create": lambda: L.smc_batch_create(None, ctypes.byref(vp)),
        "smc_batch_add": lambda: L.smc_batch_add(None, None, 10, 1, ctypes.byref(i)),
        "smc_batch_tick": lambda: L.smc_batch_tick(None, 1),
        "smc_batch_set_workgroup": lambda: L.smc_batch_set_workgroup(None, 0, 128),
        "smc_batch_set_owned": lambda: L.smc_batch_set_owned(None, 0, 1),
        "smc_batch_poll": lambda: L.smc_batch_poll(None, 0, None, None, None, None),
        "smc_batch_retire": lambda: L.smc_batch_retire(None, 0),
        "smc_resample_weights": lambda: L.smc_resample_weights(None, None, 10, 1, 0, None, None),
        "smc_resample_weights_noalloc": lambda: L.smc_resample_weights_noalloc(None, None, 10, 1, 0, None, None),
    }


def test_every_entry_point_rejects_null_handles(library):
    """NULL handles and output pointers are reported as SMC_ERR_INVALID with a
    message, before any device call; the destroy calls accept NULL."""
    from paper_2112_00364_amd import smc
    L = smc.lib()
    for name, call in _null_calls(L).items():
        assert call() == smc.ERR_INVALID, name
        assert L.smc_last_error(), name
    assert L.smc_model_destroy(None) == smc.OK
    assert L.smc_batch_destroy(None) == smc.OK


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2112_00364_amd import smc
    monkeypatch.setattr(smc, "_lib", None)
    monkeypatch.setattr(smc, "LIB_PATH", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError):
        smc.lib()


def test_stale_library_check_watches_every_source():
    """sources_newer_than_lib() (which decides whether the tests rebuild) must
    look at every source and header the library is compiled from."""
    from paper_2112_00364_amd import build as B
    on_disk = sorted(f for f in os.listdir(B.CSRC) if f.endswith((".hip", ".hpp", ".h")))
    assert sorted(B.SOURCES + B.HEADERS) == on_disk
