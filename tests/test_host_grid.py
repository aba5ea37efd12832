"""The library's grid of an array of frequencies (resolvent_grid_from_omegas: host code in the C ABI, no GPU):
the snapped spacing satisfies |domega| P h = 2 pi with P the multiple of the stride nearest the array's own
period (the time grid of Sec. 2.3 holds whole periods of every analysis frequency), and malformed arrays are
refused."""
import numpy as np
import pytest


def _lib_or_skip():
    from paper_2008_10904_amd import _lib
    try:
        return _lib.load()
    except (ImportError, OSError) as e:  # the library is not built in this checkout
        pytest.skip("libresolvent.so not loadable: %s" % e)


@pytest.mark.parametrize("w0,w1,n,h,stride", [
    (-3.0, 3.0, 256, 0.001, 256),   # the GL periodic workload's band, projected every 256th step
    (-2.0, 2.0, 64, 0.01, 1),
    (0.0, np.pi / 2, 96, 0.1, 38),
    (2.0, -2.0, 33, 0.05, 1),       # descending
])
def test_grid_from_omegas_snaps_to_whole_periods(w0, w1, n, h, stride):
    _lib_or_skip()
    from paper_2008_10904_amd.api import grid_from_omegas
    w = np.linspace(w0, w1, n)
    g, P = grid_from_omegas(w, h, stride)
    dw_nom = (w1 - w0) / (n - 1)
    assert g.n_omega == n and g.omega0 == w[0]
    assert P % stride == 0 and P >= n
    assert abs(abs(g.domega) * P * h - 2 * np.pi) < 1e-12 * 2 * np.pi
    assert np.sign(g.domega) == np.sign(dw_nom)
    # nearest multiple of the stride: neither neighbour is closer to the array's own period
    per = 2 * np.pi / (abs(dw_nom) * h)
    for Q in (P - stride, P + stride):
        if Q >= 1:
            assert abs(per - P) <= abs(per - Q) + 1e-9


def test_grid_from_omegas_errors():
    _lib_or_skip()
    from paper_2008_10904_amd import ResolventError
    from paper_2008_10904_amd import _lib as L
    from paper_2008_10904_amd.api import grid_from_omegas
    w = np.linspace(-1, 1, 20)
    bad = w.copy()
    bad[7] += 1e-4
    cases = [(w[:1], 0.01, 1, L.RES_EGRID),                 # one frequency fixes no spacing
             (bad, 0.01, 1, L.RES_EGRID),                   # off the uniform grid
             (np.zeros(4), 0.01, 1, L.RES_EGRID),           # equal end points
             (np.array([0.0, np.nan, 2.0]), 0.01, 1, L.RES_EGRID),
             (w, 0.0, 1, L.RES_EINVAL),                      # h <= 0
             (w, 0.01, 0, L.RES_EINVAL),                     # stride < 1
             (np.linspace(-100, 100, 50), 0.5, 1, L.RES_EGRID),  # P = 2 steps for 50 frequencies: aliasing
             (np.array([0.0, 1e-17]), 1.0, 1 << 40, L.RES_EGRID)]   # a period beyond any step count
    for arr, h, stride, code in cases:
        with pytest.raises(ResolventError) as e:
            grid_from_omegas(arr, h, stride)
        assert e.value.code == code
