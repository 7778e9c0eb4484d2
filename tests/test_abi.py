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


def test_struct_layouts_match_the_c_header(tmp_path):
    """sizeof / offsetof of every struct of include/automat.h, compiled as C,
    against the ctypes mirrors of the binding."""
    import os
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    inc = os.path.join(os.path.dirname(__file__), "..", "include")
    checks = {
        "automat_phase": ("Phase", ["kind", "E", "nu", "H", "sigma_y", "sigma0", "eps0", "n"]),
        "automat_params": ("Params", ["n_phases", "phase"]),
        "automat_ms_options": ("MsOptions", ["tol", "max_iter", "fixed_iter", "lambda0", "mu0",
                                             "newton_tol", "newton_max_iter", "ref_update",
                                             "warm_start", "reserved"]),
        "automat_request": ("Request", [f[0] for f in _lib.Request._fields_]),
        "automat_result": ("Result", [f[0] for f in _lib.Result._fields_]),
        "automat_server_stats_t": ("ServerStats", [f[0] for f in _lib.ServerStats._fields_]),
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "automat.h"', "int main(void) {"]
    for cname, (_, fields) in checks.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fields:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", f"-I{inc}", str(src), "-o", str(exe)], check=True)
    got = {}
    for line in subprocess.run([str(exe)], check=True, capture_output=True,
                               text=True).stdout.splitlines():
        parts = line.split()
        got[tuple(parts[:-1])] = int(parts[-1])
    for cname, (pyname, fields) in checks.items():
        cls = getattr(_lib, pyname)
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in fields:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
