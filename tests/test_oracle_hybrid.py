"""Pins of the oracle's Hybrid Gridding and column pruning (Algorithm "The
studied Hybrid Gridding Algorithm", Section 2.4.4; Convolution-Based FFT
Pruning, Algorithm of Section 2.5.2; the Column Pruner's output equation,
Section 7.1.1), independent of the oracle's own code:

* hybrid gridding followed by column pruning with the gridding kernel itself
  (S_z = 2S, alpha = beta/2) samples exactly what the (already pinned)
  convolutional gridder computes: output row 2k equals grid row k, bit for
  bit with dyadic taps and integer visibilities  -> u taps, v nearest pixel,
  pruning offsets, kernel orientation and the half-open footprint;
* the nearest fine row and the u footprint of single records match an exact
  rational enumeration of the rect and support intervals, ties included;
* a delta pruning kernel decimates; a general one equals a circular
  convolution evaluated with numpy's FFT (the convolution theorem), then
  decimated  -> pruning indices, wrap-around, coefficient order;
* linearity, and a window equals the slice of the full grid.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import Geometry
from tests.test_oracle_pins import _brute_axis


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def _sym_dyadic_taps(beta, S, rng):
    """A symmetric table of beta S + 1 dyadic values with zero end taps."""
    h = beta * S // 2
    half = rng.integers(-8, 9, h + 1) / 8.0
    t = np.concatenate([half[:0:-1], half])       # t[h + d] = half[|d|]
    assert t.shape[0] == beta * S + 1 and np.array_equal(t, t[::-1])
    t[0] = t[-1] = 0.0
    return t


@pytest.mark.parametrize("beta,S", [(4, 7), (8, 7), (6, 4), (4, 1)])
def test_hybrid_then_prune_with_the_kernel_equals_convolutional_gridding(beta, S):
    rng = _rng(beta * 100 + S)
    nu, nv = 40, 36
    taps = _sym_dyadic_taps(beta, S, rng)
    g = Geometry(nu=nu, nv=nv, beta=beta, scale_u=1.0, scale_v=1.0, support=S)
    nrec = 400
    # records whose convolutional footprint lies inside the grid, so the
    # pruner's circular wrap reaches none of them; a few on exact ties
    pos = rng.uniform(S / 2 + 1, np.array([nu, nv]) - S / 2 - 1, (nrec, 2))
    pos[:40, 1] = (np.round(pos[:40, 1] * beta) + 0.5) / beta
    uvw = np.concatenate([pos - np.array([nu // 2, nv // 2]), np.zeros((nrec, 1))], 1)
    vis = rng.integers(-4, 5, (nrec, 2)) + 1j * rng.integers(-4, 5, (nrec, 2))
    conv, sk = oracle.grid(g, taps, uvw, vis)
    assert sk == 0
    hy, sk2 = oracle.hybrid_grid(g, taps, uvw, vis)
    assert sk2 == 0 and hy.shape == (2, beta * nv, nu)
    alpha = beta // 2 if beta >= 2 else 1
    pruned = oracle.prune_columns(hy, alpha, taps, 2 * S)
    assert pruned.shape == (2, beta * nv // alpha, nu)
    assert np.array_equal(pruned[:, ::2, :], conv)
    assert np.abs(conv).max() > 0


@pytest.mark.parametrize("beta,S", [(8, 7), (4, 6), (3, 4), (2, 1)])
def test_hybrid_single_records_match_rational_enumeration(beta, S):
    rng = _rng(7 + beta)
    n = 32
    taps = rng.uniform(0.5, 1.5, beta * S + 1)          # all non-zero
    g = Geometry(nu=n, nv=n, beta=beta, scale_u=1.0, scale_v=1.0, support=S)
    xs = list(rng.uniform(S / 2 + 1, n - S / 2 - 1, (60, 2)))
    xs += [np.array([(q + 0.5) / beta, (q + 0.5) / beta]) for q in range(beta * 4, beta * 9, 3)]
    for x in xs:
        uvw = np.array([[x[0] - n // 2, x[1] - n // 2, 0.0]])
        hy, sk = oracle.hybrid_grid(g, taps, uvw, np.array([[1.0 + 0j]]))
        assert sk == 0
        _, cells, tap_idx, ok = _brute_axis(float(x[0]), n, beta, S)
        qv, _, _, _ = _brute_axis(float(x[1]), n, beta, S)
        assert ok
        want = np.zeros((beta * n, n))
        want[qv, cells] = taps[tap_idx]
        assert np.array_equal(hy[0].real, want), x
        assert not hy[0].imag.any()


def test_hybrid_skips_out_of_range_and_non_finite_records():
    g = Geometry(nu=16, nv=16, beta=4, scale_u=1.0, scale_v=1.0, support=4)
    taps = np.ones(17)
    uvw = np.array([[0.0, 0.0, 0.0], [np.nan, 0, 0], [0, np.inf, 0], [-7.6, 0, 0],
                    [0.0, -8.2, 0.0], [0.0, 7.8, 0.0], [5.5, 0.0, 0.0], [0.0, 7.9, 0.0]])
    hy, sk = oracle.hybrid_grid(g, taps, uvw, np.ones((8, 1)))
    # kept: the centre and u = 5.5 (row 32, cells 7..10 and 12..15), v = 7.8
    # (row floor(4 * 15.8 + 1/2) = 63, the last); skipped: NaN, Inf, u = -7.6
    # (first cell -1), v = -8.2 (row -1), v = 7.9 (row 64)
    assert sk == 5
    assert hy[0, 63].real.sum() == 4 and hy[0, 32].real.sum() == 8


def test_prune_with_a_delta_kernel_decimates():
    rng = _rng(3)
    x = rng.standard_normal((2, 48, 5)) + 1j * rng.standard_normal((2, 48, 5))
    for alpha, Sz in ((4, 6), (3, 2), (1, 4)):
        z = np.zeros(alpha * Sz + 1)
        z[alpha * Sz // 2] = 1.0
        assert np.array_equal(oracle.prune_columns(x, alpha, z, Sz), x[:, ::alpha, :])


@pytest.mark.parametrize("alpha,Sz", [(4, 14), (2, 6), (3, 4), (8, 16)])
def test_prune_equals_fft_circular_convolution_then_decimation(alpha, Sz):
    rng = _rng(alpha * 31 + Sz)
    M = alpha * 24
    x = rng.standard_normal((3, M, 7)) + 1j * rng.standard_normal((3, M, 7))
    z = rng.standard_normal(alpha * Sz + 1)
    got = oracle.prune_columns(x, alpha, z, Sz)
    # out[j] = sum_d c(d) x[alpha j + d] = (x circularly convolved with h)[alpha j],
    # h[(-d) mod M] = c(d), d in [-alpha Sz/2, alpha Sz/2)
    h = np.zeros(M)
    for d in range(-alpha * Sz // 2, alpha * Sz // 2):
        h[(-d) % M] += z[d + alpha * Sz // 2]
    y = np.fft.ifft(np.fft.fft(x, axis=1) * np.fft.fft(h)[None, :, None], axis=1)
    want = y[:, ::alpha, :]
    assert np.linalg.norm(got - want) / np.linalg.norm(want) < 1e-13


def test_hybrid_linearity_and_window():
    rng = _rng(5)
    g = Geometry(nu=30, nv=20, beta=8, scale_u=0.9, scale_v=1.1, support=7)
    taps = rng.standard_normal(57)
    uvw = np.concatenate([rng.uniform(-14, 14, (300, 1)), rng.uniform(-9, 9, (300, 1)),
                          np.zeros((300, 1))], 1)
    x = rng.standard_normal((300, 3)) + 1j * rng.standard_normal((300, 3))
    y = rng.standard_normal((300, 3)) + 1j * rng.standard_normal((300, 3))
    a, b = 0.5 - 1j, 2.0 + 0.25j
    Gx, _ = oracle.hybrid_grid(g, taps, uvw, x)
    Gy, _ = oracle.hybrid_grid(g, taps, uvw, y)
    Gxy, _ = oracle.hybrid_grid(g, taps, uvw, a * x + b * y)
    assert np.allclose(Gxy, a * Gx + b * Gy, rtol=0, atol=1e-12 * np.abs(Gxy).max())
    Gw, _ = oracle.hybrid_grid(g, taps, uvw, x, window=(3, 17, 11, 40))
    assert np.array_equal(Gw, Gx[:, 17:57, 3:14])
