"""Pins for the grid diffusion oracle (oracle/stencil.py): a point-by-point
version with explicit bounds checks, the exact spread of a single point,
uniform fields (interior unchanged, edges and corners losing the share of
their missing neighbours), conservation, linearity and the grid's
symmetries."""
import numpy as np
import pytest

from oracle import stencil as S


@pytest.mark.parametrize("shape", [(1, 1), (1, 7), (5, 1), (3, 4), (9, 13)])
def test_vectorised_equals_point_by_point(shape):
    rng = np.random.default_rng(shape[0] * 31 + shape[1])
    c = rng.random(shape)
    for D in (0.0, 0.1, 0.5, 1.0):
        assert np.allclose(S.diffuse(c, D), S.diffuse_loops(c, D), rtol=0, atol=1e-15)


def test_single_point_spreads_to_its_eight_neighbours():
    c = np.zeros((7, 9))
    c[3, 4] = 1.0
    D = 0.2
    out = S.diffuse(c, D)
    want = np.zeros_like(c)
    want[2:5, 3:6] = D / 8
    want[3, 4] = 1 - D
    assert np.array_equal(out, want)
    assert out.sum() == pytest.approx(1.0)


def test_uniform_field_loses_mass_only_at_the_border():
    u, D = 2.0, 0.4
    out = S.diffuse(np.full((6, 8), u), D)
    assert np.allclose(out[1:-1, 1:-1], u)
    assert out[0, 0] == pytest.approx((1 - D) * u + D / 8 * 3 * u)     # corner: 3 neighbours
    assert out[0, 3] == pytest.approx((1 - D) * u + D / 8 * 5 * u)     # edge: 5 neighbours
    # total mass lost = D/8 * sum over points of value * (number of missing neighbours)
    miss = np.zeros((6, 8))
    for y in range(6):
        for x in range(8):
            miss[y, x] = sum(1 for dy in (-1, 0, 1) for dx in (-1, 0, 1)
                             if (dy or dx) and not (0 <= y + dy < 6 and 0 <= x + dx < 8))
    assert out.sum() == pytest.approx(6 * 8 * u - D / 8 * u * miss.sum())


def test_linearity_and_symmetries():
    rng = np.random.default_rng(2)
    a, b = rng.random((11, 17)), rng.random((11, 17))
    D = 0.3
    assert np.allclose(S.diffuse(2 * a + 3 * b, D), 2 * S.diffuse(a, D) + 3 * S.diffuse(b, D))
    assert np.allclose(S.diffuse(a.T, D), S.diffuse(a, D).T)
    assert np.allclose(S.diffuse(a[::-1, ::-1], D), S.diffuse(a, D)[::-1, ::-1])
    assert np.array_equal(S.diffuse(a, 0.0), a)
    assert np.allclose(S.diffuse(a, D, steps=3), S.diffuse(S.diffuse(S.diffuse(a, D), D), D))
