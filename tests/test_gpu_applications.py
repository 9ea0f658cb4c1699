"""The paper's application integrands (Sec. 4.5-4.6) compiled at run time and
integrated on the GPU, against their closed forms (tests/closed_forms.py,
pinned by quadrature in test_applications.py): FP64 sample path, 5
iterations not combined, then 10 combined; the estimate within 4 sigma of
the closed form (the payoff's lognormal tail makes the per-iteration
variance estimates noisy) and its relative error estimate below the stated
bound."""
import math
import sys

import numpy as np
import pytest

from tests import closed_forms as cf

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def run(src, dim, params, lo, hi, n_g, n_eval):
    from paper_2408_09229_amd import UserIntegrand, Vegas, make_config
    fn = UserIntegrand(src, dim, "f64")
    v = Vegas(make_config(dim, n_g, n_eval, precision="f64"), 0, params, lo, hi, user=fn)
    v.adapt(5)
    v.integrate(10)
    r = v.result()
    v.close()
    fn.close()
    return r.integral, math.sqrt(r.sigma2)


def test_asian_call():
    from paper_2408_09229_amd import integrands
    p = integrands.asian_params()
    exact = cf.asian_call(p, 8)
    I, s = run(integrands.ASIAN_CALL, 8, p, np.zeros(8), np.ones(8), 1024, 1_000_000)
    say(f"[asian] {I:.6f} +- {s:.2e} exact {exact:.6f} z {(I - exact) / s:.2f}")
    assert abs(I - exact) < 4.0 * s
    assert s < 2e-3 * exact


@pytest.mark.parametrize("xe", [0.0, 1.0])
def test_feynman_ho(xe):
    from paper_2408_09229_amd import integrands
    p = integrands.feynman_params(x_end=xe, t=4.0, n=8)
    lo, hi = integrands.feynman_box(8)
    exact = cf.feynman_ho(p, 7)
    I, s = run(integrands.FEYNMAN_HO, 7, p, lo, hi, 256, 1_000_000)
    say(f"[feynman x={xe}] {I:.6f} +- {s:.2e} exact {exact:.6f} z {(I - exact) / s:.2f}")
    assert abs(I - exact) < 4.0 * s
    assert s < 1e-3 * exact
