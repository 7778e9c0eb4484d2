"""The C-ABI library loads and exports every symbol its header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2006_04391_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(automat_\w+)\s*\(", text))
    return names


def test_header_declares_entry_points():
    names = _declared_functions()
    assert {"automat_evaluate", "automat_evaluate_ex", "automat_evaluate_backward"} <= names


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in sorted(_declared_functions()) if not hasattr(L, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH), reason="library not built")
def test_host_only_entry_points():
    L = _lib.load()
    assert L.automat_version().decode().startswith("automat")
    assert L.automat_strerror(-1).decode() == "invalid argument"
    for name in _lib.SIGNATURES:
        assert hasattr(L, name), name


def test_param_struct_layout_matches_header():
    # automat_phase: int32 kind, int32 reserved, 7 doubles
    assert ctypes.sizeof(_lib.Phase) == 8 + 7 * 8
    assert ctypes.sizeof(_lib.Params) == 8 + _lib.MAX_PHASES * ctypes.sizeof(_lib.Phase)
    p = _lib.make_params([dict(kind=1, E=1.0, nu=0.3, H=0.0, sigma_y=0.0, sigma0=1.0, eps0=1.0,
                               n=2.0)])
    assert p.n_phases == 1 and p.phase[0].nu == 0.3
    with pytest.raises(ValueError):
        _lib.make_params([])


def test_product_path_has_no_cpu_fallback():
    """The binding refuses CPU tensors instead of computing on the host."""
    torch = pytest.importorskip("torch")
    from paper_2006_04391_amd import api, inputs
    ps = inputs.points_c0(n=8)
    t = lambda x: torch.from_numpy(x)
    with pytest.raises((ValueError, RuntimeError)):
        api.evaluate(t(ps.eps), t(ps.a_old), t(ps.phase), ps.phases)


def test_package_does_not_import_oracle():
    """Only tests, the smoke check and the benchmark's CPU leg touch the oracle."""
    pkg = os.path.join(ROOT, "paper_2006_04391_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "oracle_" not in text, fn
