"""How far the oracle's operator arithmetic moves the results.

The oracle scales every operator by the reciprocal of its fixed metric
divisor (1/d_e, 1/l_e, 1/A_c, 1/A_v, 1/valence, 1/3), formed once as the IEEE
quotient 1/x.  The operators' plain statement divides: the divergence and
curl are (1/A) times a sum, the gradients a difference over a length, the
averages a sum over a count.  Both readings are the same mathematics and
differ only in rounding.  This test builds a second oracle with the literal
divisions in every such place and runs the recipe cases of the flat R2B4x20
workload and an R2B4x30 terrain case for 10 steps under both, reporting each
field's max-relative departure.  The kernels follow the reciprocal reading,
so their bitwise agreement with the oracle holds for that reading; this test
measures what the other reading would change.  CPU only."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

from oracle import build as OB

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nhdc_oracle.c")
FIELDS = ("vn", "w", "rho", "pi", "theta_v")


def literal_division_source(src):
    """The oracle's source with each `x * (1.0 / d)` of a fixed metric divisor
    d written as `x / (d)`, and each cell-area reciprocal `ia` likewise.  The
    sponge factor 1/(1 + dt r) is a multiplication by definition and stays."""
    out, pos, n = [], 0, 0
    key = " * (1.0 / "
    while True:
        i = src.find(key, pos)
        if i < 0:
            out.append(src[pos:])
            break
        j, depth = i + len(key), 1
        while depth:
            depth += {"(": 1, ")": -1}.get(src[j], 0)
            j += 1
        operand = src[i + len(key):j - 1]
        if operand.startswith("(1.0 + dt"):
            out.append(src[pos:j])
        else:
            out.append(src[pos:i] + " / (" + operand + ")")
            n += 1
        pos = j
    res = "".join(out)
    res, m = re.subn(r"double ia = 1\.0 / g->cell_area\[c\];", "const double ia = g->cell_area[c];", res)
    res, m2 = re.subn(r"\] \* ia;", "] / ia;", res)
    return res, n, m, m2


# the child runs one case for 10 steps with the oracle build named by ORACLE_SO
CHILD = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
from paper_2511_02021_amd.inputs import case as CS
which, out = sys.argv[2], sys.argv[3]
c = CS.config_case(1) if which == "flat" else CS.config_case(2, k=4, n_lev=30)
m = oracle.Model(c)
for _ in range(10):
    m.step(c.dt, c.nsub)
s = m.state()
facc, wacc = m.flux()
np.savez(out, facc=facc, wacc=wacc, **{k: s[k] for k in ("vn", "w", "rho", "pi", "theta_v")})
"""


@pytest.fixture(scope="module")
def builds(tmp_path_factory):
    d = tmp_path_factory.mktemp("division")
    src, n, m, m2 = literal_division_source(open(SRC).read())
    assert n >= 15 and m == 2 and m2 == 2, (n, m, m2)
    (d / "nhdc_oracle.c").write_text(src)
    so_div = str(d / "liboracle_division.so")
    r = subprocess.run(OB.command(str(d / "nhdc_oracle.c"), so_div), capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    so_rec = OB.SO if os.path.exists(OB.SO) else OB.build()
    return d, {"reciprocal": so_rec, "division": so_div}


def _run(d, so, which, label):
    out = str(d / f"{which}_{label}.npz")
    env = dict(os.environ, ORACLE_SO=so, OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS", "8"))
    r = subprocess.run([sys.executable, "-c", CHILD, ROOT, which, out], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    return np.load(out)


def test_literal_division_source_is_the_same_mathematics():
    src, n, _, _ = literal_division_source(open(SRC).read())
    assert " * (1.0 / g->" not in src and " * (1.0 / 3.0)" not in src
    assert "wp[i] * (1.0 / (1.0 + dt * p->w_damp[i]))" in src
    # on exact numbers the two readings agree: x * (1/d) = x / d for d = 4, 8
    assert 3.0 * (1.0 / 4.0) == 3.0 / 4.0 and 5.0 * (1.0 / 8.0) == 5.0 / 8.0


@pytest.mark.parametrize("which", ["flat", "terrain"])
def test_departure_of_the_literal_division_reading(builds, which):
    """Every field of the two readings after 10 steps.  Measured: flat R2B4x20
    departs by 3.4e-12 in w, 1.2e-12 in the vertical mass flux and at most
    1.5e-13 elsewhere; the R2B4x30 terrain case by 3.1e-11 in w, 2.6e-12 in
    the vertical mass flux and at most 1.8e-13 elsewhere.  So w and its flux
    are above 1e-12: the kernels' bitwise agreement with the oracle in w rests
    on their sharing the reciprocal reading."""
    d, so = builds
    a = _run(d, so["reciprocal"], which, "reciprocal")
    b = _run(d, so["division"], which, "division")
    dep = {}
    for f in FIELDS + ("facc", "wacc"):
        dep[f] = float(np.abs(a[f] - b[f]).max() / np.abs(a[f]).max())
    print(f"\n{which}: max-relative departure of the literal-division reading after 10 steps: "
          + ", ".join(f"{f} {v:.2e}" for f, v in dep.items()))
    assert dep["vn"] > 0.0  # the readings do round differently
    w_bar = 1e-11 if which == "flat" else 1e-10
    assert dep["w"] <= w_bar, dep
    for f in ("vn", "rho", "pi", "theta_v", "facc"):
        assert dep[f] <= 1e-12, (f, dep)
    assert dep["wacc"] <= w_bar, dep
