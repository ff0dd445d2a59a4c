"""The C-ABI library loads and exports every function include/air.h declares (no GPU needed)."""
import ctypes
import os

import pytest

from paper_2108_07001_amd import air


def test_header_declares_the_boundary():
    names = air.header_functions()
    for required in ["air_create", "air_destroy", "air_const_create", "air_const_destroy",
                     "air_llr", "air_mi_gmi", "air_sweep", "air_sync", "air_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(air.LIB_PATH), "build libair.so first (python -m paper_2108_07001_amd.build)"
    lib = ctypes.CDLL(air.LIB_PATH)
    missing = [n for n in air.header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_create_rejects_bad_device_without_gpu_work():
    lib = air.load()
    h = ctypes.c_void_p()
    assert lib.air_create(ctypes.byref(h), -1, None) == air.AIR_E_INVAL
    assert lib.air_create(None, 0, None) == air.AIR_E_INVAL
    # every entry point tolerates a null context
    assert lib.air_sync(None) == air.AIR_E_INVAL
    assert lib.air_llr(None, None, None, 1, 0.0, 1, None) == air.AIR_E_INVAL
    assert lib.air_mi_gmi(None, None, None, None, 1, 0.0, 1, None, None) == air.AIR_E_INVAL
    assert lib.air_sweep(None, None, None, None, 1, None, 1, 1, None, None) == air.AIR_E_INVAL
    assert lib.air_llr_aux(None, None, None, 1, 1.0, 1, None) == air.AIR_E_INVAL
    assert lib.air_mi_gmi_aux(None, None, None, None, 1, 1.0, 1, None, None) == air.AIR_E_INVAL
    assert lib.air_noise_var(None, None, None, None, 1, 1, None) == air.AIR_E_INVAL
    assert lib.air_const_bits(None) == 0
    lib.air_destroy(None)
    lib.air_const_destroy(None)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    monkeypatch.setattr(air, "_lib", None)
    monkeypatch.setattr(air, "LIB_PATH", str(tmp_path / "libair.so"))
    with pytest.raises(RuntimeError):
        air.load()


def test_q_factor_matches_oracle():
    """air_q_factor_db is host arithmetic: checked here without a GPU."""
    import math
    import oracle
    from paper_2108_07001_amd import air
    for ber in (1e-6, 1e-4, 3.8e-3, 2e-2, 0.1, 0.3):
        assert abs(air.q_factor_db(ber) - oracle.q_factor_db(ber)) < 1e-9
    assert math.isnan(air.q_factor_db(0.0)) and math.isnan(air.q_factor_db(0.5))
