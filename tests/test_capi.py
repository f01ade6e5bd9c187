"""The C ABI library loads and exports every function include/*.h declares (no GPU needed)."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        src = open(h).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"\b(pisco_[a-z0-9_]+)\s*\(", src):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["pisco_create", "pisco_destroy", "pisco_set_sky", "pisco_set_beam", "pisco_set_detector",
                 "pisco_set_pointing", "pisco_convolve", "pisco_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_1908_05662_amd import _lib

    lib = _lib.load()
    missing = [n for n in sorted(_declared()) if not hasattr(lib, n)]
    assert not missing, missing
    assert lib.pisco_abi_version() == 100


def test_binding_covers_every_declared_symbol():
    from paper_1908_05662_amd import _lib

    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert _declared() <= bound, sorted(_declared() - bound)


def test_create_without_gpu_fails_cleanly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    from paper_1908_05662_amd import _lib

    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.pisco_create(0, ctypes.byref(h)) != _lib.OK
    assert lib.pisco_last_error(None) == b"null context"
    # every entry point rejects a null context instead of crashing
    assert lib.pisco_set_sky(None, 64, None, None, None, 0, 0) == _lib.EINVAL
    assert lib.pisco_convolve(None, 0, 0, None, 0, None) == _lib.EINVAL
    assert lib.pisco_output_samples(None, 0) == -1


def test_no_cpu_fallback_in_product_path():
    """The product package never imports the oracle."""
    for p in glob.glob(os.path.join(ROOT, "paper_1908_05662_amd", "**", "*.py"), recursive=True):
        src = open(p).read()
        assert "import oracle" not in src and "from oracle" not in src, p


def test_spectra_host_logic():
    from paper_1908_05662_amd import _lib

    lib = _lib.load()
    assert lib.pisco_alm_size(10) == 66 and lib.pisco_alm_size(0) == 1 and lib.pisco_alm_size(-1) == 0
    nalm = 192 * 193 // 2
    partial = 8 * nalm * 6 * 8                        # per-wave partial sums of the a_lm
    it = 12 * 64 * 64 * 8 + nalm * 16                 # per field: residual map and a_lm correction
    assert lib.pisco_map2alm_workspace_bytes(64, 191, 1) == 3 * 192 * 255 * 16 + partial + 3 * it
    assert lib.pisco_map2alm_workspace_bytes(64, 191, 0) == 192 * 255 * 16 + partial + it
    assert lib.pisco_map2alm_workspace_bytes(48, 10, 1) == -1       # not a power of two
    assert lib.pisco_map2alm_workspace_bytes(2048, 10, 1) == -1     # above the largest nside
    assert lib.pisco_map2alm_workspace_bytes(8, 33, 1) == -1        # lmax above 4 nside
    assert lib.pisco_map2alm(None, 8, 10, 0, None, None, None, None, None, None, None, 0, None) == _lib.EINVAL
    assert lib.pisco_alm2map(None, 8, 10, None, None, None, None, None, None, None, 0, None) == _lib.EINVAL
    assert lib.pisco_anafast(None, 8, 10, 0, None, None, None, None, None, None, None, 0, None, None) == _lib.EINVAL
    assert lib.pisco_alm2cl(None, 10, None, None, None, None) == _lib.EINVAL
