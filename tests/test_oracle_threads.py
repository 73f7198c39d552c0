"""The oracle's parallel cell loops change nothing: results with several
threads are bitwise those of one thread (only loops whose iterations write
disjoint outputs run in parallel; every sum keeps its serial order).  Also
the lifetime of the C model behind a stepper: a stepper made from a model
object that the caller drops must keep that model alive (a use after free
here crashed a GPU smoke run once; under the sanitizer build this test
reports it)."""
import gc

import numpy as np

import oracle as O
from synth import fields as F
from synth.mesh import get_mesh


def _run(threads):
    O.set_threads(threads)
    try:
        m = get_mesh(3)
        s = O.SWE(m)
        u0 = F.initial_state("c1_exprb42_l4", level=3)
        rng = np.random.default_rng(5)
        v = rng.standard_normal(s.N)
        out = [s.rhs(u0), s.jv(u0, v), s.jtv(u0, v)]
        st = O.swe_stepper(s, "exprb53")
        u = u0
        for _ in range(2):
            u = st.step(u, 1800.0)
        out.append(u)
        W, _, _ = s.phi_combo(u0, 900.0, [None, v * 1e-3, None, v * 1e-4], [0.5, 1.0])
        out += W
        return out
    finally:
        O.set_threads(1)


def test_threads_bitwise():
    a = _run(1)
    b = _run(4)
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def test_stepper_keeps_its_model_alive():
    m = get_mesh(2)
    u0 = F.initial_state("c1_exprb42_l4", level=2)
    st = O.swe_stepper(O.SWE(m), "exprb42")   # the model object is not kept here
    gc.collect()
    got = st.step(u0, 900.0)
    ref = O.swe_stepper(O.SWE(m), "exprb42").step(u0, 900.0)
    assert np.array_equal(got, ref)
