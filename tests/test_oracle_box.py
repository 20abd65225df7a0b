"""Pins for the oracle's routines on boxes of nx x ny x nz cells (the
definition with a separate length per axis, and the convolution with each
axis padded to twice its own length), against facts fixed outside them:
an independent FFT library on non-cubic arrays, the box sum itself, the
exact impulse response (the kernel), the reduction to the already pinned
routines on cubes, an axis permutation with unequal lengths, and the
monopole far field.  Arrays are [z][y][x].
"""
import math

import numpy as np
import pytest

from paper_2409_02294_amd import inputs


def _box_density(shape, seed):
    rng = np.random.default_rng(seed)
    nz, ny, nx = shape
    z, y, x = np.meshgrid((np.arange(nz) + 0.5) / nz, (np.arange(ny) + 0.5) / ny, (np.arange(nx) + 0.5) / nx,
                          indexing="ij")
    rho = np.zeros(shape)
    for _ in range(3):
        c = rng.uniform(0.3, 0.7, 3)
        s = rng.uniform(0.08, 0.15)
        rho += rng.uniform(0.5, 2.0) * np.exp(-((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) / (2 * s * s))
    return rho + 1e-3 * rng.uniform(0, 1, shape)


@pytest.mark.parametrize("shape", [(4, 6, 10), (12, 5, 8), (9, 16, 3), (1, 7, 2)])
def test_fft3_box_matches_numpy(oracle_lib, shape):
    rng = np.random.default_rng(sum(shape))
    a = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    for sign, ref in ((-1, np.fft.fftn(a)), (+1, np.fft.ifftn(a) * a.size)):
        got = oracle_lib.fft3_box(a, sign)
        assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("shape,sp", [((6, 10, 8), (0.1, 0.13, 0.07)), ((8, 4, 12), (1 / 12, 1 / 12, 1 / 12)),
                                      ((5, 9, 3), (0.2, 0.05, 0.11)), ((1, 1, 6), (0.3, 0.3, 0.3))])
def test_box_fft_conv_equals_direct_sum(oracle_lib, shape, sp):
    rho = _box_density(shape, 11)
    a = oracle_lib.direct_sum_box(rho, *sp, G=0.7)
    b = oracle_lib.fft_conv_box(rho, *sp, G=0.7)
    assert oracle_lib.rel_l2(b, a) <= 1e-13
    cells = [(0, 0, 0), (shape[0] - 1, shape[1] - 1, shape[2] - 1), (shape[0] // 2, shape[1] // 3, shape[2] // 2)]
    c = oracle_lib.direct_sum_cells_box(rho, cells, *sp, G=0.7)
    assert np.allclose(c, [a[z, y, x] for z, y, x in cells], rtol=1e-15, atol=0)


def test_box_routines_reduce_to_the_cube_routines(oracle_lib):
    # on a cube the box routines compute what the (separately pinned) cubic
    # routines compute, with equal and with unequal spacings
    n = 10
    rho = inputs.make_density(n, 4, 91, sigma=(0.05, 0.12))
    for sp in ((0.1, 0.1, 0.1), (0.1, 0.25, 0.4)):
        assert oracle_lib.rel_l2(oracle_lib.fft_conv_box(rho, *sp), oracle_lib.fft_conv3(rho, *sp)) <= 1e-14
        assert oracle_lib.rel_l2(oracle_lib.direct_sum_box(rho, *sp), oracle_lib.direct_sum3(rho, *sp)) <= 1e-15
        kb = oracle_lib.kernel_pad_box(n, n, n, *sp)
        assert np.array_equal(kb, oracle_lib.kernel_pad3(n, *sp))


@pytest.mark.parametrize("c", [(0, 0, 0), (5, 2, 9), (6, 7, 11)])
def test_box_impulse_response_is_the_kernel(oracle_lib, c):
    # a unit mass in cell c: phi[i] = G K(i - c) exactly, K from its closed
    # definition on dx x dy x dz cells (including the self cell of a box)
    shape, (dx, dy, dz) = (7, 8, 12), (0.1, 0.17, 0.06)
    rho = np.zeros(shape)
    rho[c] = 1.0 / (dx * dy * dz)
    phi = oracle_lib.fft_conv_box(rho, dx, dy, dz, G=1.5)
    z, y, x = np.meshgrid(*[np.arange(s) for s in shape], indexing="ij")
    ref = 1.5 * np.vectorize(lambda a, b, cc: oracle_lib.kernel_value3(cc - c[2], b - c[1], a - c[0], dx, dy, dz))(
        z, y, x)
    assert np.abs(phi - ref).max() <= 1e-14 * np.abs(ref).max()


def test_box_axis_permutation(oracle_lib):
    # exchanging the x and z axes of a box (lengths and spacings with them)
    # transposes the potential; so does cycling all three axes
    shape, sp = (6, 10, 14), (0.07, 0.1, 0.13)  # (nz, ny, nx), (dx, dy, dz)
    rho = _box_density(shape, 21)
    a = oracle_lib.fft_conv_box(rho, *sp)
    b = oracle_lib.fft_conv_box(np.ascontiguousarray(np.transpose(rho, (2, 1, 0))), sp[2], sp[1], sp[0])
    assert oracle_lib.rel_l2(np.transpose(b, (2, 1, 0)), a) <= 1e-14
    # (z, y, x) -> (y, x, z): new x is old z, new y is old x, new z is old y
    c = oracle_lib.fft_conv_box(np.ascontiguousarray(np.transpose(rho, (1, 2, 0))), sp[2], sp[0], sp[1])
    assert oracle_lib.rel_l2(np.transpose(c, (2, 0, 1)), a) <= 1e-14


def test_box_kernel_pad_is_even_per_axis(oracle_lib):
    nx, ny, nz, sp = 5, 3, 4, (0.1, 0.2, 0.3)
    k = oracle_lib.kernel_pad_box(nx, ny, nz, *sp)
    assert k.shape == (2 * nz, 2 * ny, 2 * nx)
    for axis in range(3):
        p = k.shape[axis]
        idx = (-np.arange(p)) % p
        assert np.array_equal(np.take(k, idx, axis=axis), k)
    assert k[0, 0, 0] == oracle_lib.kernel_value3(0, 0, 0, *sp)
    assert k[1, 2, 3] == oracle_lib.kernel_value3(3, 2, 1, *sp)
    assert k[7, 5, 9] == oracle_lib.kernel_value3(1, 1, 1, *sp)


def test_box_monopole_far_field(oracle_lib):
    # a compact blob in an elongated box: at the far corners phi -> -G M / r
    nz, ny, nx = 12, 20, 40
    dx = dy = dz = 1 / 40
    zc, yc, xc = (np.arange(nz) + 0.5) * dz, (np.arange(ny) + 0.5) * dy, (np.arange(nx) + 0.5) * dx
    z, y, x = np.meshgrid(zc, yc, xc, indexing="ij")
    cz, cy, cx = zc[nz // 2], yc[ny // 2], xc[4]
    s = 0.02
    rho = np.exp(-((x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2) / (2 * s * s))
    mass = rho.sum() * dx * dy * dz
    phi = oracle_lib.fft_conv_box(rho, dx, dy, dz)
    for (a, b, c) in [(0, 0, nx - 1), (nz - 1, ny - 1, nx - 1), (0, ny - 1, nx - 2)]:
        r = math.sqrt((z[a, b, c] - cz) ** 2 + (y[a, b, c] - cy) ** 2 + (x[a, b, c] - cx) ** 2)
        assert abs(phi[a, b, c] + mass / r) <= 2e-3 * mass / r
