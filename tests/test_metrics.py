"""The oscillation metrics of the pulsed point-source check, on fields whose
answer is known by construction."""
import numpy as np

from bench import oscillation_metrics, p_lattice_from_torn


def _bump(n, shift=0.0):
    x = np.linspace(0.0, 1.0, n + 1)
    X, Y = np.meshgrid(x, x)
    return (np.exp(-((X - 0.5) ** 2 + (Y - 0.5) ** 2) / 0.02) + shift).ravel()


def test_smooth_bump_has_one_extremum_per_midline_and_no_undershoot():
    und, cnt = oscillation_metrics(_bump(16), 16)
    assert und == 0.0 and cnt == 2


def test_negative_dip_is_measured_as_undershoot():
    p = _bump(16, shift=-0.1)
    und, _ = oscillation_metrics(p, 16)
    assert abs(und - 0.1 / 0.9) < 1e-9  # the bump itself adds exp(-25) at the corners


def test_checkerboard_adds_extrema():
    n = 16
    p = _bump(n).reshape(n + 1, n + 1)
    cb = 0.05 * ((np.add.outer(np.arange(n + 1), np.arange(n + 1)) % 2) * 2 - 1)
    _, cnt = oscillation_metrics((p + cb).ravel(), n)
    assert cnt > 10


def test_nan_outside_the_region_is_ignored():
    n = 16
    p = _bump(n).reshape(n + 1, n + 1)
    p[:, :4] = np.nan
    und, cnt = oscillation_metrics(p.ravel(), n)
    assert und == 0.0 and cnt == 2


def test_p_lattice_from_torn_places_pressure_dofs():
    codes = np.array([8 * 3 + 4, 8 * 3 + 0, 8 * 5 + 4, 8 * 3 + 4])
    u = np.array([1.5, 9.0, -2.0, 1.5])
    lat = p_lattice_from_torn(codes, u, 2)
    assert lat[3] == 1.5 and lat[5] == -2.0 and np.isnan(lat[0])
