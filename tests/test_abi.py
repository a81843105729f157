"""C-ABI checks that need no GPU: the library loads, exports every entry
point declared in include/pm.h, validates parameters, and its host-side mask
generator matches the shared input generator bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_0802_2488_amd import _lib, synth
from paper_0802_2488_amd.solver import make_params

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z0-9_]+)\s*\(", txt)))


def test_header_symbols_exported():
    names = _declared()
    assert len(names) >= 12
    L = _lib.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(n for n, _, _ in _lib.SIGNATURES) == names


def test_workspace_bytes_and_validation():
    L = _lib.lib()
    p = make_params(64, precision="fp64")
    n64 = L.pm_workspace_bytes(ctypes.byref(p))
    p32 = make_params(64, precision="fp32")
    n32 = L.pm_workspace_bytes(ctypes.byref(p32))
    # stress state (4 planes) and 3-component half spectrum dominate
    assert n64 > 4 * 64 * 64 * 8 + 64 * 33 * 48
    assert n32 < n64
    for bad in (make_params(48), make_params(2), make_params(16384), make_params(64, mu=-1.0),
                make_params(64, Y=0.0), make_params(64, max_iter=0), make_params(64, green_variant=6),
                make_params(64, mu0=-1.0)):
        assert L.pm_workspace_bytes(ctypes.byref(bad)) == 0
        assert b"" != L.pm_last_error()


def test_status_strings_and_tile():
    L = _lib.lib()
    assert L.pm_status_string(0) == b"ok"
    assert L.pm_status_string(-4).startswith(b"not converged")
    for n in (4, 64, 4096, 8192):
        for prec in (0, 1):
            WT = L.pm_spectrum_tile(n, prec)
            assert WT >= 1 and (n // 2) % WT == 0
    assert L.pm_spectrum_tile(48, 0) < 0
    assert L.pm_spectrum_tile(64, 3) < 0


def test_create_rejects_bad_arguments_without_touching_the_device():
    L = _lib.lib()
    h = ctypes.c_void_p()
    p = make_params(64)
    assert L.pm_solver_create(ctypes.byref(h), ctypes.byref(p), None, None, 0, None) == _lib.PM_EINVAL
    p_bad = make_params(100)
    assert L.pm_solver_create(ctypes.byref(h), ctypes.byref(p_bad), 256, 256, 1 << 30, None) == _lib.PM_EINVAL
    # misaligned workspace
    assert L.pm_solver_create(ctypes.byref(h), ctypes.byref(p), 256, 260, 1 << 30, None) == _lib.PM_EINVAL
    # too small workspace
    assert L.pm_solver_create(ctypes.byref(h), ctypes.byref(p), 256, 256, 16, None) == _lib.PM_EINVAL


@pytest.mark.parametrize("L,f,seed", [(1, 0.5, 0), (17, 0.3, 5), (64, 0.1, 0), (128, 0.4, 1234567)])
def test_host_mask_matches_shared_generator(L, f, seed):
    buf = np.zeros(L * L, np.uint8)
    rc = _lib.lib().pm_bernoulli_mask(buf.ctypes.data, L, f, seed, 0, None)
    assert rc == 0
    np.testing.assert_array_equal(buf.reshape(L, L), synth.bernoulli_mask(L, f, seed))


def test_mask_porosity_statistics():
    m = synth.bernoulli_mask(512, 0.3, 0)
    assert abs(m.mean() - 0.3) < 4 * np.sqrt(0.3 * 0.7 / m.size)
    assert synth.bernoulli_mask(64, 0.0, 1).sum() == 0
    assert synth.bernoulli_mask(64, 1.0, 1).sum() == 64 * 64


@pytest.mark.parametrize("L,f", [(64, 0.1), (128, 0.1), (256, 0.3)])
def test_circular_void_cell(L, f):
    m = synth.circular_void(L, f)
    assert m.dtype == np.uint8 and m.shape == (L, L)
    # area within the pixels crossed by the boundary circle
    assert abs(int(m.sum()) - f * L * L) <= 2 * np.pi * L * np.sqrt(f / np.pi) + 4
    # symmetric under both mirrors and the transpose of the cell
    assert np.array_equal(m, m[::-1, :]) and np.array_equal(m, m[:, ::-1]) and np.array_equal(m, m.T)
    # one 4-connected cluster
    from scipy import ndimage
    assert ndimage.label(m)[1] == 1


def test_missing_library_fails_loudly(tmp_path):
    """Without libpm.so the product path raises: there is no fallback."""
    import subprocess
    import sys

    code = (
        "from paper_0802_2488_amd import _lib\n"
        "try:\n"
        "    _lib.lib()\n"
        "except RuntimeError as e:\n"
        "    assert 'missing' in str(e), e\n"
        "    print('raised')\n"
        "else:\n"
        "    raise SystemExit('no error')\n"
        "import numpy as np\n"
        "from paper_0802_2488_amd import solver\n"
        "try:\n"
        "    solver.Solver(np.zeros((8, 8), np.uint8), solver.make_params(8))\n"
        "except RuntimeError:\n"
        "    print('raised')\n"
        "else:\n"
        "    raise SystemExit('solver built without the library')\n"
    )
    env = dict(os.environ, PM_LIB_PATH=str(tmp_path / "absent" / "libpm.so"))
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                         timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.split() == ["raised", "raised"]
