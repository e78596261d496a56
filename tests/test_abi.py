"""C-ABI library: loads, exports every declared symbol, host-side logic (CPU only)."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import riem
from paper_2604_20384_amd.inputs import make_problem, num_gates, random_antihermitian

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "qhvp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(qhvp_[a-z0-9_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_2604_20384_amd import _lib
    names = _declared_functions()
    assert len(names) >= 18
    for name in names:
        assert hasattr(_lib.lib, name), name
    raw = ctypes.CDLL(_lib.LIB_PATH)
    for name in names:
        getattr(raw, name)


def test_num_gates_matches_layout():
    from paper_2604_20384_amd import api
    for n in range(2, 25):
        for L in range(1, 12):
            assert api.num_gates(n, L) == num_gates(n, L)
    assert api.num_gates(1, 3) == -1 and api.num_gates(4, 0) == -1


def test_workspace_bytes():
    from paper_2604_20384_amd import api
    S = 256 * 2 ** 20 * 8
    w1 = api.workspace_bytes(20, 20, 40, 256, "c64", ckpt_every=1, with_tangent=True)
    w0 = api.workspace_bytes(20, 20, 40, 256, "c64", ckpt_every=0, with_tangent=True)
    w4 = api.workspace_bytes(20, 20, 40, 256, "c64", ckpt_every=4, with_tangent=True)
    wg = api.workspace_bytes(20, 20, 40, 256, "c64", ckpt_every=1, with_tangent=False)
    assert w0 > w1 > S and w4 < w1
    assert wg < w1
    assert api.workspace_bytes(20, 20, 40, 256, "c128", 1, True) > 1.9 * w1
    assert api.workspace_bytes(1, 20, 40, 256, "c64", 1, True) == 0
    assert api.workspace_bytes(20, 20, 40, 0, "c64", 1, True) == 0


def test_projection_and_riemannian_hvp_match_oracle():
    from paper_2604_20384_amd import api
    p = make_problem(2, 9, 1, seed=12)
    rng = np.random.default_rng(0)
    K = p.K
    X = rng.standard_normal((K, 4, 4)) + 1j * rng.standard_normal((K, 4, 4))
    gr = rng.standard_normal((K, 4, 4)) + 1j * rng.standard_normal((K, 4, 4))
    H = rng.standard_normal((K, 4, 4)) + 1j * rng.standard_normal((K, 4, 4))
    V = p.G @ random_antihermitian(rng, K)
    assert np.allclose(api.project(p.G, X), riem.project(p.G, X), atol=1e-15)
    assert np.allclose(api.riemannian_hvp(p.G, gr, H, V), riem.riemannian_hvp(p.G, gr, H, V), atol=1e-14)
    assert api.unitarity_error(p.G) < 1e-14
    assert api.unitarity_error(p.G + 1e-3) > 1e-4


def test_retraction_matches_polar_factor():
    from paper_2604_20384_amd import api
    p = make_problem(2, 7, 1, seed=13)
    rng = np.random.default_rng(1)
    xi = p.G @ random_antihermitian(rng, p.K)
    for t in (0.0, 1e-3, 0.5, 2.0):
        R = api.retract(p.G, t * xi)
        assert np.allclose(R, riem.retract(p.G, t * xi), atol=1e-13)
        assert api.unitarity_error(R) < 1e-13


def test_errors_are_reported_not_raised_in_c():
    from paper_2604_20384_amd import _lib
    from paper_2604_20384_amd._lib import QhvpError, check, lib
    with pytest.raises(QhvpError):
        check(lib.qhvp_project(0, None, None, None))
    assert "bad arguments" in lib.qhvp_last_error().decode()
    h = ctypes.c_void_p()
    st = lib.qhvp_ctx_create(10 ** 6, ctypes.byref(h))      # no such device (or no GPU at all)
    assert st in (_lib.QHVP_ERR_INVALID, _lib.QHVP_ERR_DEVICE)
    assert lib.qhvp_overlaps(None, None, None) == _lib.QHVP_ERR_INVALID
    assert lib.qhvp_hvp_batch(None, None, 1, None, 0, None, None, None) == _lib.QHVP_ERR_INVALID
    assert lib.qhvp_states_kept_for(None, None) == -1


def test_product_path_has_no_fallback():
    """The binding imports nothing from the oracle and refuses to run without the library."""
    import subprocess
    import sys
    code = ("import os; os.environ['QHVP_LIB']='/nonexistent/libqhvp.so'\n"
            "try:\n import paper_2604_20384_amd._lib\nexcept ImportError as e: print('IMPORTERROR', e)\n")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=ROOT)
    assert "IMPORTERROR" in r.stdout
    pkg = os.path.join(ROOT, "paper_2604_20384_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith(".py"):
                txt = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", txt, flags=re.M), f
