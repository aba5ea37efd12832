"""The library's FIR design (resolvent_fir_design: host code in the C ABI, no GPU) against the oracle's, and its
argument errors."""
import numpy as np
import pytest

from oracle import trm as O_trm


def _lib_or_skip():
    from paper_2008_10904_amd import _lib
    try:
        return _lib.load()
    except (ImportError, OSError) as e:  # the library is not built in this checkout
        pytest.skip("libresolvent.so not loadable: %s" % e)


@pytest.mark.parametrize("order,nu,gain", [
    (40, [-1.0, 1.0], [1.0, 1.0]),
    (200, list(np.linspace(-1, 1, 41)), list(np.exp(-(np.linspace(-1, 1, 41) / 0.3) ** 2))),
    (600, [-1.0, -0.2, -0.05, 0.1, 0.19, 0.3, 1.0], [0.0, 0.0, 1e-3, 0.4, 1.0, 0.0, 0.0]),
    (1030, [-0.5, 0.25], [2.0, 0.5]),   # held at the end values outside the breakpoints; grid of 2 * 2048
])
def test_fir_design_matches_oracle(order, nu, gain):
    _lib_or_skip()
    from paper_2008_10904_amd.api import fir_design
    got = fir_design(order, nu, gain)
    ref = O_trm.fir_design(order, np.array(nu), np.array(gain))
    assert np.abs(got - ref).max() < 1e-12 * max(np.abs(ref).max(), 1e-300)


def test_fir_design_errors():
    _lib_or_skip()
    from paper_2008_10904_amd import ResolventError
    from paper_2008_10904_amd import _lib as L
    from paper_2008_10904_amd.api import fir_design
    for order, nu, gain in ((41, [-1, 1], [1, 1]), (0, [-1, 1], [1, 1]), (40, [0.5, -0.5], [1, 1]),
                            (40, [-1, 1], [1, -1]), (40, [-1.5, 1], [1, 1]), (40, [0.0], [1.0])):
        with pytest.raises(ResolventError) as e:
            fir_design(order, nu, gain)
        assert e.value.code == L.RES_EINVAL
