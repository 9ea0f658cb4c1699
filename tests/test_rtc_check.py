"""Integrands compiled at run time: the library's embedded device headers and
a caller's source compile for gfx950 with hipRTC (no device needed), and a
source that does not compile is rejected with the compiler's log.  CPU only."""
import pytest

ROOS_F64 = """
__device__ vegas_real vegas_user_f(const vegas_real* x, int dim, const double* p)
{
    vegas_real r = (vegas_real)p[0];
    for (int d = 0; d < dim; ++d) r *= fabs((vegas_real)4 * x[d] - (vegas_real)2);
    return r;
}
"""


@pytest.fixture(scope="module")
def pk():
    import paper_2408_09229_amd as pk
    return pk


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_user_source_compiles(pk, prec):
    pk.UserIntegrand.check(ROOS_F64, 5, prec)


def test_syntax_error_reported(pk):
    bad = "__device__ vegas_real vegas_user_f(const vegas_real* x, int dim, const double* p) { return x[0] +; }"
    with pytest.raises(pk.VegasError) as e:
        pk.UserIntegrand.check(bad, 3, "f64")
    assert e.value.status == pk.abi.VEGAS_EINVAL
    assert "error" in str(e.value)


def test_missing_function_reported(pk):
    with pytest.raises(pk.VegasError) as e:
        pk.UserIntegrand.check("__device__ double g(double x) { return x; }", 3, "f64")
    assert "vegas_user_f" in str(e.value)


@pytest.mark.parametrize("dim,prec", [(0, "f64"), (17, "f64")])
def test_bad_arguments(pk, dim, prec):
    with pytest.raises(pk.VegasError) as e:
        pk.UserIntegrand.check(ROOS_F64, dim, prec)
    assert e.value.status == pk.abi.VEGAS_EINVAL
