"""vegas_create_static: a context whose workspace is the library's own device
array (for callers that cannot allocate), against vegas_create on a caller
workspace.  Two static contexts in a row, the second on a smaller problem,
each checked against a context on a torch workspace with the same inputs.

The first pair runs the FP32 sample path with FP64 accumulators (the hot
fill kernel).  Its first iteration's estimate, variance and allocation come
from per-cube sums taken in a fixed order, so they are compared bit for bit;
the map is compared at 1e-12 relative (its histogram bins are LDS atomic
sums, whose rounding follows the order of the adds); the later iterations
and the combined result at 1e-12 relative.  The second pair runs ORDERED
accumulation in FP64, where the whole trajectory is bit for bit.
"""
import numpy as np
import pytest

import vegas_inputs as vi

pytestmark = pytest.mark.gpu


def _make(w, accum, static):
    from paper_2408_09229_amd import Vegas, make_config
    cfg = make_config(w.dim, w.n_g, w.n_eval, alpha=w.alpha, beta=w.beta, seed=w.seed, precision=w.precision,
                      accum=accum, max_iter=16)
    return Vegas(cfg, w.family, w.params, static=static)


def _snapshot(v):
    I, s2 = v.get_iterations()
    return I, s2, v.get_nh(), v.get_map()


def _pair(w, accum):
    import torch
    torch.cuda.set_device(0)
    a = _make(w, accum, static=True)
    b = _make(w, accum, static=False)
    assert a.ws is None and b.ws is not None
    a.adapt(1)
    b.adapt(1)
    first = (_snapshot(a), _snapshot(b))
    a.integrate(2)
    b.integrate(2)
    last = (_snapshot(a), _snapshot(b))
    ra, rb = a.result(), b.result()
    a.close()
    b.close()
    return first, last, (ra, rb)


def test_static_matches_workspace_then_smaller():
    from paper_2408_09229_amd import make_config, workspace_size
    from paper_2408_09229_amd import abi
    big = vi.gauss3_8d().with_(n_eval=2_000_003, n_g=256)
    small = vi.gauss_prod_4d().with_(n_eval=20_011, n_g=32)
    sizes = []
    for w, acc in ((big, "fp64"), (small, "ordered")):
        cfg = make_config(w.dim, w.n_g, w.n_eval, alpha=w.alpha, beta=w.beta, seed=w.seed,
                          precision=w.precision, accum=acc, max_iter=16)
        sizes.append(workspace_size(cfg, w.family, w.params))
    assert sizes[1] < sizes[0] <= abi.STATIC_SCRATCH_BYTES, sizes

    # first call: the larger problem, FP32 samples, FP64 accumulators
    (fa, fb), (la, lb), (ra, rb) = _pair(big, "fp64")
    assert np.array_equal(fa[0], fb[0]) and np.array_equal(fa[1], fb[1]), (fa[:2], fb[:2])
    assert np.array_equal(fa[2], fb[2])
    np.testing.assert_allclose(fa[3], fb[3], rtol=1e-12, atol=0)
    assert len(la[0]) == len(lb[0]) == 3
    np.testing.assert_allclose(la[0], lb[0], rtol=1e-12, atol=0)
    np.testing.assert_allclose(la[1], lb[1], rtol=1e-12, atol=0)
    assert ra.n_iter_combined == rb.n_iter_combined == 2
    assert abs(ra.integral - rb.integral) <= 1e-12 * abs(rb.integral)
    assert abs(ra.sigma2 - rb.sigma2) <= 1e-12 * rb.sigma2

    # second call: a smaller problem in the same array, ORDERED: bit for bit
    (fa, fb), (la, lb), (ra, rb) = _pair(small, "ordered")
    for x, y in zip(fa + la, fb + lb):
        assert np.array_equal(x, y)
    assert (ra.integral, ra.sigma2, ra.chi2_dof) == (rb.integral, rb.sigma2, rb.chi2_dof)


def test_static_rejects_oversized_problem():
    from paper_2408_09229_amd import Vegas, VegasError, make_config, workspace_size
    from paper_2408_09229_amd import abi
    w = vi.gauss3_8d()          # 1e8 samples, 1024 intervals: far beyond the array
    cfg = make_config(w.dim, w.n_g, w.n_eval, alpha=w.alpha, beta=w.beta, seed=w.seed, precision=w.precision)
    assert workspace_size(cfg, w.family, w.params) > abi.STATIC_SCRATCH_BYTES
    with pytest.raises(VegasError) as e:
        Vegas(cfg, w.family, w.params, static=True)
    assert e.value.status == abi.VEGAS_ENOMEM
