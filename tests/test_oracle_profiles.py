"""Pins of the oracle's profile and observable definitions (no GPU): level
crossings of linear profiles are exact, sentinels and the highest / outermost
choice, sums, and the contact line of a constructed half-frozen drop."""

import numpy as np

from oracle import profiles as PR


def test_column_top_is_exact_on_linear_profiles():
    ny, nx = 40, 3
    y = np.arange(ny, dtype=float)[:, None]
    h = np.array([12.3, 0.25, 30.9])
    v = 0.5 + 0.1 * (h[None, :] - y)
    assert np.abs(PR.column_top(v) - h).max() < 1e-12


def test_column_top_sentinels_and_highest_region():
    v = np.zeros((10, 3))
    v[9, 0] = 0.7              # top row itself
    v[2:4, 1] = 1.0            # two regions: the higher one counts
    v[6, 1] = 0.8
    top = PR.column_top(v)
    assert top[0] == 9.0
    assert abs(top[1] - (6 + 0.3 / 0.8)) < 1e-12
    assert top[2] == -1.0


def test_row_edges_on_ramps_and_sentinels():
    nx = 30
    x = np.arange(nx, dtype=float)
    a, b = 7.4, 21.8
    tri = np.minimum(0.5 + 0.2 * (x - a), 0.5 + 0.2 * (b - x))
    v = np.stack([tri, np.zeros(nx), np.ones(nx)])
    left, right = PR.row_edges(v)
    assert abs(left[0] - a) < 1e-12 and abs(right[0] - b) < 1e-12
    assert left[1] == -1.0 and right[1] == -1.0
    assert left[2] == 0.0 and right[2] == nx - 1


def test_sums_and_solid_fraction():
    rng = np.random.default_rng(0)
    fs = rng.uniform(0, 1, (6, 5))
    chi = np.maximum(fs, rng.uniform(0, 1, (6, 5)))
    p = PR.profiles({"fs": fs, "chi": chi})
    assert np.allclose(p["col"]["ice"], [sum(fs[y, x] for y in range(6)) for x in range(5)])
    assert np.allclose(p["row"]["pcm"], [sum(chi[y, x] for x in range(5)) for y in range(6)])
    assert abs(PR.solid_fraction(p) - fs.sum() / chi.sum()) < 1e-14


def test_contact_line_of_a_constructed_drop():
    """Half-disc of material (radius 10) above row 4, frozen up to row 4 + 6
    inclusive: the contact line is at height 6, half-width the chord there."""
    ny, nx, R, base, H = 24, 40, 10.0, 4, 6
    yy, xx = np.mgrid[0:ny, 0:nx].astype(float)
    chi = (((xx - 20.0) ** 2 + (yy - base) ** 2 < R * R) & (yy >= base)).astype(float)
    fs = chi * (yy <= base + H)
    p = PR.profiles({"fs": fs, "chi": chi})
    R_tr, H_tr = PR.contact_line(p, base)
    assert H_tr == H
    row = chi[base + H]
    xs = np.nonzero(row)[0]
    assert abs(R_tr - 0.5 * ((xs[-1] + 0.5) - (xs[0] - 0.5))) < 1e-12
    assert PR.contact_line(PR.profiles({"fs": 0 * chi, "chi": chi}), base) is None
