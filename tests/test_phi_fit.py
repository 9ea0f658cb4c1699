"""The warp's FP32 Gaussian distribution function and its inverse
(flow_dev.hpp: phi_lower, phi_inv_lower): their coefficients are the ones
csrc/fit_phi.py fits, and that FP32 operation sequence, emulated on the
host, stays within its stated error against scipy in FP64."""
import os
import re
import sys

import numpy as np
import pytest
from scipy.special import ndtr, ndtri

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_2408_09229_amd", "csrc")
sys.path.insert(0, CSRC)
import fit_phi  # noqa: E402


def device_polys():
    """The Horner coefficients of each polynomial in phi_lower and
    phi_inv_lower, in source order (highest degree first)."""
    src = open(os.path.join(CSRC, "flow_dev.hpp")).read()
    out = []
    for fn in ("phi_lower", "phi_inv_lower"):
        body = src[src.index(f"float {fn}("):]
        body = body[:body.index("\n}\n")]
        for m in re.finditer(r"(\w) = (-?[\d.]+e[-+]\d+)f;((?:\s+\1 = fmaf\(\1, \w, -?[\d.]+e[-+]\d+f\);)+)", body):
            coefs = [float(m.group(2))] + [float(v) for v in re.findall(r"(-?[\d.]+e[-+]\d+)f\);", m.group(3))]
            out.append(np.array(coefs, np.float32))
    return out


@pytest.fixture(scope="module")
def fits():
    c1, c2 = fit_phi.fit_inverse()
    return {"central": c1, "tail": c2, "lower": fit_phi.fit_lower()}


def test_device_coefficients_are_the_fit(fits):
    lower, central, tail = device_polys()
    assert np.array_equal(lower, fits["lower"])
    assert np.array_equal(central, fits["central"])
    assert np.array_equal(tail, fits["tail"])


def test_lower_tail_error(fits):
    a = fit_phi.r32(np.linspace(0, 12, 200001))
    r = np.abs(fit_phi.phi_lower32(fits["lower"], a) / ndtr(-a.astype(np.float64)) - 1)
    assert r.max() < 7 * 2.0 ** -24
    # a = 0 gives 1/2 to the same few ulps, and the tail decreases
    h = fit_phi.phi_lower32(fits["lower"], np.array([0.0, 1.0, 2.0, 4.0, 8.0]))
    assert abs(h[0] - 0.5) < 4 * 2.0 ** -25 and np.all(np.diff(h) < 0)


def test_inverse_error(fits):
    m = np.logspace(-7, np.log10(0.4999), 200000)
    w = -np.log(4 * m * (1 - m))
    p = np.where(w < 5.0, fit_phi.horner32(fits["central"], fit_phi.r32(w - 2.5)),
                 fit_phi.horner32(fits["tail"], fit_phi.r32(np.sqrt(w) - 3)))
    r = np.abs(-np.sqrt(2) * p.astype(np.float64) * (1 - 2 * m) / ndtri(m) - 1)
    assert r.max() < 4 * 2.0 ** -24
