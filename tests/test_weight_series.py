"""The edge-weight series of the LDS-staged product (host logic, no GPU).

The product forms the flux weight alpha = c (a/2) asin(y)/y and the
circulation weight beta = alpha (1 - y^2)^(-1/2) from the edge's Laplacian
weight c and the half-chord y between the two unit centres, each factor a
truncated series in y^2; the host gives a grid chunk tables (and with them
the LDS product) only when every edge lies in the series' range, and picks
four terms instead of five on grids whose half-chords are short enough.
These tests pin the series' coefficients to the functions they sum, bound
the truncation remainders at the two thresholds in 50-digit arithmetic, check
that the host's and the kernels' thresholds are the same numbers, and check
on which side of them the icosahedral grids of levels 6-8 fall."""
import math
import os
import re
from decimal import Decimal, getcontext

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_02144_amd", "csrc")


def series_coefficients(nterms):
    """asin(y)/y = sum a_k y^(2k) and (1 - y^2)^(-1/2) = sum b_k y^(2k)."""
    a, b = [Decimal(1)], [Decimal(1)]
    for k in range(nterms - 1):
        a.append(a[-1] * (2 * k + 1) ** 2 / ((2 * k + 2) * (2 * k + 3)))
        b.append(b[-1] * (2 * k + 1) / (2 * k + 2))
    return a, b


def constant(path, name):
    text = open(os.path.join(CSRC, path)).read()
    m = re.search(r"constexpr\s+(?:double|int)\s+%s\s*=\s*([0-9.eE+-]+)\s*;" % name, text)
    assert m, "%s not found in %s" % (name, path)
    return float(m.group(1))


def remainders(y2, nterms, total=60):
    """Sums of the omitted terms (k >= nterms) of both series at y^2, in 50 digits."""
    getcontext().prec = 50
    a, b = series_coefficients(total)
    y2 = Decimal(repr(y2))
    ra = sum(a[k] * y2 ** k for k in range(nterms, total))
    rb = sum(b[k] * y2 ** k for k in range(nterms, total))
    return float(ra), float(rb)


def test_coefficients_sum_to_the_functions():
    getcontext().prec = 50
    a, b = series_coefficients(80)
    for y in (0.05, 0.2, 0.4):
        y2 = Decimal(repr(y)) ** 2
        fa = float(sum(c * y2 ** k for k, c in enumerate(a)))
        fb = float(sum(c * y2 ** k for k, c in enumerate(b)))
        # the library functions are within an ulp or so of the true values
        assert fa == pytest.approx(math.asin(y) / y, rel=3e-16, abs=0)
        assert fb == pytest.approx(1.0 / math.sqrt(1.0 - y * y), rel=3e-16, abs=0)


def test_remainders_at_the_thresholds():
    nt = int(constant("stencil_common.h", "kShortTerms"))
    y5 = constant("stencil_common.h", "kShortY2Max")
    y4 = constant("stencil_common.h", "kShort4Y2Max")
    assert nt == 5
    # both factors are near 1, so these are relative errors of alpha and beta
    ra, rb = remainders(y5, nt)
    assert ra < 3e-18 and rb < 3e-18, (ra, rb)
    ra, rb = remainders(y4, 4)
    assert ra < 3e-19 and rb < 3e-19, (ra, rb)
    # one term fewer at either threshold would not be exact to rounding
    assert max(remainders(y5, nt - 1)) > 1e-16
    assert max(remainders(y4, 3)) > 1e-16


def test_host_and_kernel_thresholds_agree():
    assert constant("geometry.cpp", "kShortY2MaxHost") == constant("stencil_common.h", "kShortY2Max")
    assert constant("geometry.cpp", "kShort4Y2MaxHost") == constant("stencil_common.h", "kShort4Y2Max")


@pytest.mark.parametrize("level,terms", [(6, 5), (7, 4), (8, 4)])
def test_grid_ranges(level, terms):
    from synth.mesh import get_mesh
    m = get_mesh(level)
    x = np.asarray(m["xyz"], dtype=np.float64)
    nb = np.asarray(m["nbr"])
    d = x[nb] - x[:, None, :]
    y2max = float((0.25 * (d * d).sum(-1)).max())
    assert y2max <= constant("geometry.cpp", "kShortY2MaxHost")
    four = y2max <= constant("geometry.cpp", "kShort4Y2MaxHost")
    assert (4 if four else 5) == terms, y2max
