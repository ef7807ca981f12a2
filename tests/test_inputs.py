"""The seeded inputs: the slab-by-slab generator of the shell (for grids
too large to hold whole) gives exactly the planes of the whole-grid one,
and the fv quadrature does not depend on how its cells are batched."""
import numpy as np

from paper_1810_13416_amd import problems as pr


def test_shell_planes_equal_the_whole_grid():
    n = 24
    full = pr.config3(n=n)
    assert pr.config3_params(n) == full.params
    for k0, nk in ((0, 5), (5, 11), (16, 8), (23, 1)):
        sl = pr.config3_planes(n, k0, nk)
        for q in range(15):
            assert np.array_equal(sl[q], full.state[q][k0:k0 + nk]), (k0, q)


def test_fv_quadrature_is_independent_of_the_chunk_size():
    P = pr.config3_params(16)
    ball = lambda X, Y, Z: (X * X + Y * Y + Z * Z >= 0.25).astype(np.float64)
    a = pr.fv_moments_quadrature(P, ball, chunk=1 << 16)
    b = pr.fv_moments_quadrature(P, ball, chunk=37)
    for q in range(10):
        assert np.array_equal(a[q], b[q]), q
