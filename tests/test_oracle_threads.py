"""The reference's element loops run on several threads (OpenMP); its results
do not depend on the thread count, bit for bit (every value is computed by the
same arithmetic in the same order)."""
import numpy as np

import oracle as O
from paper_2305_13847_amd import synth


def _runs(case, **over):
    o = O.Oracle.for_case(case, **over)
    R = o.rhs(case.U)
    U1, out = o.rk(case.U, case.dt, 2)
    return R, U1, out, o.mass(case.U)


def test_results_do_not_depend_on_the_thread_count():
    cases = [(synth.warm_rain_3d(n=(4, 3, 3), order=3, seed=5), {}),
             (synth.moist_bubble(n=(6, 4), order=2, seed=6), {"sip_gamma": 0.3})]
    try:
        for case, over in cases:
            O.set_threads(1)
            a = _runs(case, **over)
            O.set_threads(4)
            b = _runs(case, **over)
            for x, y in zip(a, b):
                assert np.array_equal(np.asarray(x), np.asarray(y))
    finally:
        O.set_threads(0)
