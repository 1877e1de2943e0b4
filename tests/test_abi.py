"""Host-side checks of the C ABI: the library loads, exports every function
that include/treepm.h declares, and rejects invalid parameters without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "treepm.h")
LIB = os.path.join(ROOT, "paper_1909_04667_amd", "libtreepm.so")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(tpm_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_operations():
    names = _declared()
    for n in ("tpm_build_tree", "tpm_compute_forces", "tpm_pm_long_range", "tpm_create",
              "tpm_destroy", "tpm_export_tree"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(LIB)
    for n in _declared():
        assert hasattr(L, n), n


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_parameter_validation_on_host():
    from paper_1909_04667_amd import binding as B
    L = B.lib()
    ok = B.make_params(eps=0.01)
    assert L.tpm_bytes_needed(ctypes.byref(ok), 1000) > 0
    iso = B.make_params(eps=0.01, pm_grid=64)  # isolated TreePM
    assert L.tpm_bytes_needed(ctypes.byref(iso), 1000) > L.tpm_bytes_needed(ctypes.byref(ok), 1000)
    bad = [dict(eps=0.0), dict(eps=0.01, alpha=0.0), dict(eps=0.01, theta=-1.0),
           dict(eps=0.01, periodic=True, box_size=10.0),                 # no mesh
           dict(eps=0.01, periodic=True, box_size=10.0, pm_grid=48),     # not 2^k
           dict(eps=0.01, pm_grid=512),                                  # isolated > 256
           dict(eps=0.01, pm_grid=8),                                    # isolated < 16
           dict(eps=0.01, pm_grid=64, asmth=0.0),                        # no split scale
           dict(eps=0.01, shift=(1.0, 0.0, 0.0)),
           dict(eps=0.01, periodic=True, box_size=10.0, pm_grid=8, asmth=2.0, rcut=4.5)]
    for kw in bad:
        p = B.make_params(**kw)
        assert L.tpm_bytes_needed(ctypes.byref(p), 1000) == -1, kw
        h = ctypes.c_void_p()
        assert L.tpm_create(ctypes.byref(p), None, ctypes.byref(h)) == B.TPM_EINVAL, kw
        assert not h.value
        assert L.tpm_create_arena(ctypes.byref(p), None, 1 << 20,
                                  ctypes.byref(h)) == B.TPM_EINVAL, kw
    h = ctypes.c_void_p()
    assert L.tpm_create_arena(ctypes.byref(ok), None, -1, ctypes.byref(h)) == B.TPM_EINVAL
    assert L.tpm_create_arena(ctypes.byref(ok), None, 1 << 20, None) == B.TPM_EINVAL
    # the admission estimate grows with n and covers the mesh
    sizes = [L.tpm_bytes_needed(ctypes.byref(ok), n) for n in (1, 10, 1000, 10 ** 6)]
    assert sizes == sorted(sizes) and sizes[-1] > 150 * 10 ** 6
    per = B.make_params(eps=0.01, periodic=True, box_size=10.0, pm_grid=128)
    assert L.tpm_bytes_needed(ctypes.byref(per), 1000) > 128 ** 3 * 8
    # NULL arguments are rejected before anything touches a device
    assert L.tpm_set_shift(None, None) == B.TPM_EINVAL
    assert L.tpm_build_tree(None, 10, None, None, None, None) == B.TPM_EINVAL
    assert L.tpm_compute_forces(None, 0, 1, None, None, None, None, None) == B.TPM_EINVAL
    assert L.tpm_check(None) == B.TPM_EINVAL


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_product_path_does_not_reference_the_oracle():
    """The HIP library and its binding never load the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1909_04667_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in txt and "liboracle" not in txt, f
