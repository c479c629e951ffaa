"""GPU parity of the grid diffusion step (libswstencil) against the fp64
oracle, and bit-equality of the padded and bounds-checked forms.

Tolerance: a step forms each output from 9 fp32 values with 10 roundings
(the neighbour sums, the two products) and the fp32 coefficients 1 - D and
D/8; with values in [0, 1] every step adds at most about 12 * 2^-24 < 1e-6
of absolute error, so k steps stay within 1e-6 * k."""
import numpy as np
import pytest

from oracle import stencil as S

pytestmark = pytest.mark.gpu


def run(grid, D, steps, padded):
    import torch
    from paper_2208_12350_amd import stencil as K
    g = torch.from_numpy(np.ascontiguousarray(grid, dtype=np.float32)).cuda()
    ny, nx = g.shape
    if padded:
        a = K.pad(g)
        b = a.clone()
        for _ in range(steps):
            K.diffuse_padded(a, b, nx, ny, D)
            a, b = b, a
        out = a[1:ny + 1, 1:nx + 1]
    else:
        a, b = g.clone(), torch.empty_like(g)
        for _ in range(steps):
            K.diffuse_checked(a, b, D)
            a, b = b, a
        out = a
    torch.cuda.synchronize()
    return out.cpu().numpy()


SHAPES = [(1, 1), (1, 70), (70, 1), (5, 61), (5, 62), (5, 63), (64, 124), (65, 125), (129, 200), (300, 187)]


@pytest.mark.parametrize("shape", SHAPES)
def test_one_step_matches_oracle_and_forms_agree(shape):
    rng = np.random.default_rng(shape[0] * 1000 + shape[1])
    c = rng.random(shape).astype(np.float32)
    for D in (0.0, 0.125, 0.37, 1.0):
        want = S.diffuse(c.astype(np.float64), D)
        p = run(c, D, 1, True)
        q = run(c, D, 1, False)
        assert np.array_equal(p, q)                       # same arithmetic, bounds logic aside
        assert np.max(np.abs(p - want)) <= 1e-6


def test_many_steps_and_a_point_source():
    c = np.zeros((200, 301), np.float32)
    c[0, 0] = 1.0
    c[100, 150] = 1.0
    c[199, 300] = 1.0
    steps, D = 40, 0.25
    want = S.diffuse(c.astype(np.float64), D, steps)
    p = run(c, D, steps, True)
    assert np.array_equal(p, run(c, D, steps, False))
    assert np.max(np.abs(p - want)) <= 1e-6 * steps


def test_pad_grid_layout():
    import torch
    from paper_2208_12350_amd import stencil as K
    g = torch.arange(3 * 70, dtype=torch.float32, device="cuda").reshape(3, 70) + 1
    p = K.pad(g).cpu().numpy()
    assert p.shape == (5, K.padded_pitch(70))
    assert np.array_equal(p[1:4, 1:71], g.cpu().numpy())
    p[1:4, 1:71] = 0
    assert not p.any()


def test_paper_grid_size_sampled():
    # the 2500 x 2500 held-out size of Section V-D, 10 steps
    rng = np.random.default_rng(9)
    c = rng.random((2500, 2500)).astype(np.float32)
    steps, D = 10, 0.15
    want = S.diffuse(c.astype(np.float64), D, steps)
    p = run(c, D, steps, True)
    assert np.max(np.abs(p - want)) <= 1e-6 * steps
    assert np.array_equal(p, run(c, D, steps, False))
