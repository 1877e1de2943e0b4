"""The FP64 walk's complementary error function (csrc/erfc_poly.h): the
committed coefficients reproduce erfc to 5e-15 relative for x in [0, 8]
(against 50-digit mpmath) and are what the generator writes."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1909_04667_amd", "csrc")


def _coeffs():
    txt = open(os.path.join(CSRC, "erfc_poly.h")).read()
    return [float.fromhex(h) for h in re.findall(r"^\s+(-?0x[0-9a-fA-Fp.+-]+),", txt, re.M)]


def _erfc(x, cf):
    rd = 1.0 / (4.0 + x)
    sv = (4.0 - x) * rd
    g = np.full_like(x, cf[-1])
    for c in reversed(cf[:-1]):
        g = g * sv + c
    return np.exp(-(x * x)) * ((4.0 * rd) * g)


def test_erfc_table_accuracy():
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    cf = _coeffs()
    assert len(cf) == 21
    x = np.concatenate([np.linspace(0.0, 8.0, 4001), [1e-12, 0.5, 2.25, 4.5]])
    ref = np.array([float(mp.erfc(mp.mpf(float(v)))) for v in x])
    rel = np.abs(_erfc(x, cf) - ref) / ref
    assert rel.max() <= 5e-15, rel.max()


def test_erfc_table_regenerates(tmp_path):
    pytest.importorskip("mpmath")
    src = open(os.path.join(CSRC, "erfc_poly.h")).read()
    gen = os.path.join(CSRC, "gen_erfc.py")
    work = tmp_path / "csrc"
    work.mkdir()
    (work / "gen_erfc.py").write_text(open(gen).read())
    subprocess.run([sys.executable, str(work / "gen_erfc.py")], check=True,
                   capture_output=True)
    assert (work / "erfc_poly.h").read_text() == src
