"""CPU checks of the boundary: the HIP library loads and exports every
function that include/exprb.h declares; the binding declares the same set;
the oracle and the library share no source."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "exprb.h")


def declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(xrb_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    import paper_1805_02144_amd as X
    if not os.path.exists(X.LIBPATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(X.LIBPATH)
    names = declared()
    assert len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(X.EXPORTS) == names


def test_default_params_without_gpu():
    import paper_1805_02144_amd as X
    if not os.path.exists(X.LIBPATH):
        pytest.skip("library not built")
    p = X.default_params()
    assert p.m_max == 40 and p.m_init == 1 and p.tol == 1e-10 and p.delta == 1.4
    assert p.radius == 6.371e6 and p.gravity == 9.80616


def test_oracle_and_library_share_no_source():
    csrc = os.path.join(ROOT, "paper_1805_02144_amd", "csrc")
    osrc = os.path.join(ROOT, "oracle")
    for f in os.listdir(csrc):
        txt = open(os.path.join(csrc, f)).read()
        assert "orc_" not in txt and "oracle" not in txt.lower(), f
    for f in os.listdir(osrc):
        if f.endswith((".c", ".h")):
            txt = open(os.path.join(osrc, f)).read()
            assert "xrb_" not in txt and "exprb.h" not in txt, f


def test_binding_loads_torch_before_the_library():
    """The library must bind to the HIP runtime torch loads (one runtime per
    process); the binding imports torch before it opens the library."""
    import subprocess
    import sys
    code = ("import sys, paper_1805_02144_amd as X\n"
            "assert 'torch' not in sys.modules\n"
            "X.lib()\n"
            "assert 'torch' in sys.modules\n")
    import paper_1805_02144_amd as X
    if not os.path.exists(X.LIBPATH):
        pytest.skip("library not built")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]


@pytest.mark.parametrize("cls,cname", [("Tableau", "xrb_tableau"), ("TuneResult", "xrb_tune_result")])
def test_struct_layout_matches_the_header(cls, cname):
    """The binding's ctypes structures have the size and field offsets of the
    C structs (compiled from include/exprb.h with the host C compiler)."""
    import shutil
    import subprocess
    import tempfile
    import paper_1805_02144_amd as X
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    T = getattr(X, cls)
    fields = [f[0] for f in T._fields_]
    src = ('#include <stdio.h>\n#include <stddef.h>\n#include "exprb.h"\nint main(void){\n'
           'printf("%%zu", sizeof(%s));\n' % cname +
           "".join('printf(" %%zu", offsetof(%s, %s));\n' % (cname, f) for f in fields) +
           "return 0;}\n")
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.run([cc, "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()
    got = [int(x) for x in out]
    assert got[0] == ctypes.sizeof(T)
    assert got[1:] == [getattr(T, f).offset for f in fields]


def test_scheme_tableaus_follow_the_printed_coefficients():
    """The binding's tableau encodings of exprb42, pexprb43 and exprb53 carry
    the coefficients of eqs. 3.11-3.13 (tests/golden): stage times c_i as the
    first call's output times, b_i(Z) = sum_k beta_ik phi_k(Z) as the last
    call's v_k weights of D_i, and exprb53's a_32 phi_3(c Z) terms as stage
    weights divided by c^3 (the outputs carry rho^l = c^3 on v_3)."""
    import json
    from fractions import Fraction as Fr
    import paper_1805_02144_amd as X
    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "exprb_coefficients.json")))
    for name in ("exprb42", "pexprb43", "exprb53", "exprb32"):
        T, g = X.TABLEAUS[name], gold[name]
        # internal stage times: the outputs the stages take, U_i = u_n + W(c_i)
        cs = sorted(Fr(v) for v in g["c"].values())
        first = [T.rho[0][o] for o in range(T.ns[0])]
        for c in cs:
            if c < 1:
                assert any(abs(float(c) - r) < 1e-15 for r in first), (name, c)
        # final weights: b_i's phi_k coefficient times D_i in v_k of the last call
        last = T.ncalls - 1
        for i, terms in g["b"].items():
            stage = int(i) - 2
            for k, coef in terms.items():
                k = int(k)
                assert abs(T.vc[last][k][1 + stage] - float(Fr(coef))) < 1e-12, (name, i, k)
        # exprb53: a_32 = 27/25 phi_3(Z/2) + 729/125 phi_3(9Z/10) through the
        # rho^3-weighted outputs of the second call (rho = 1/2, 9/10)
        for key, terms in g["a"].items():
            st = int(key.split(",")[0]) - 2
            for kc, coef in terms.items():
                k, c = kc.split("@")
                c = Fr(c)
                o = [T.rho[1][q] for q in range(T.ns[1])].index(float(c))
                want = Fr(coef) / c ** int(k)
                assert abs(T.uc[st][1][o] - float(want)) < 1e-12, (name, key, kc)
