"""CPU checks of the C ABI library: it loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "fciqmc.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fciqmc_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = _declared()
    for n in ["fciqmc_load_integrals", "fciqmc_init", "fciqmc_step", "fciqmc_energy",
              "fciqmc_get_walkers", "fciqmc_free_run", "fciqmc_free_system", "fciqmc_last_error"]:
        assert n in names


def test_library_exports_every_symbol():
    from paper_2006_14956_amd import fciqmc as F
    if not os.path.exists(F.LIB_PATH):
        from paper_2006_14956_amd import build
        build.build()
    lib = ctypes.CDLL(F.LIB_PATH)
    for n in _declared():
        assert hasattr(lib, n), n
    assert sorted(_declared()) == sorted(F.EXPORTS)


def test_binding_fails_loudly_without_library(monkeypatch, tmp_path):
    from paper_2006_14956_amd import fciqmc as F
    monkeypatch.setattr(F, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(F, "_lib", None)
    with pytest.raises(F.FciqmcError):
        F.lib()


def test_params_default_without_gpu():
    """fciqmc_params_default touches no device state."""
    from paper_2006_14956_amd import fciqmc as F
    if not os.path.exists(F.LIB_PATH):
        pytest.skip("library not built")
    p = F.fciqmc_params_default()
    assert p.tau == 0.01 and p.shift_interval == 10 and p.initiator_na < 0
