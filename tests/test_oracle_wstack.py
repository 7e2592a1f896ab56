"""Pins of the oracle's W-stacking (oracle/wstack.py) against what the
mathematics fixes:
  * the layer rule on exact dyadic values: layer centres, ties at the
    boundaries going up, clamping beyond the outer layers;
  * one layer at w = 0 is the plain convolutional image;
  * a point source observed with w terms (records on the layer centres and
    on the oversampled grid), W-stacked and imaged, reproduces the direct
    Fourier sum with the W-term (Section 1.7.1), while leaving out the
    layer screens or flipping the sign of the W-term does not."""
import numpy as np

import oracle
from oracle import imaging as IM
from oracle import wstack as WS
from paper_2111_04141_amd import workload as W


def test_layer_rule():
    L, dw = 5, 0.25
    centres = WS.layer_w(L, dw)
    assert np.array_equal(centres, [-0.5, -0.25, 0.0, 0.25, 0.5])
    assert np.array_equal(WS.layer_of(centres, L, 1 / dw), np.arange(L))
    # boundary between j and j + 1 at (j + 1 - L/2) dw goes up
    bounds = (np.arange(L - 1) + 1 - L / 2) * dw
    assert np.array_equal(WS.layer_of(bounds, L, 1 / dw), np.arange(1, L))
    assert np.array_equal(WS.layer_of(bounds - 1e-9, L, 1 / dw), np.arange(L - 1))
    assert np.array_equal(WS.layer_of([-100.0, 100.0], L, 1 / dw), [0, L - 1])
    # an even layer count has no layer at w = 0
    assert np.array_equal(WS.layer_w(4, 1.0), [-1.5, -0.5, 0.5, 1.5])


def test_single_layer_is_the_plain_image():
    wl = W.config_small()
    sub = W.subsample(wl.nrec, 5000, 3)
    uvw = wl.uvw[sub].astype(np.float64)
    vis = W.vis_normal(len(sub), 2, seed=4)
    geom = oracle.Geometry(nu=wl.n, nv=wl.n, beta=wl.beta, scale_u=wl.scale, scale_v=wl.scale,
                           support=wl.support)
    Gl, sk = WS.grid_layers(geom, wl.taps, uvw, vis, 1, 0.0)
    G, sk2 = oracle.grid(geom, wl.taps, uvw, vis)
    assert sk == sk2 and np.array_equal(Gl[:, 0], G)
    h = IM.corrector(wl.n, wl.beta, wl.taps, wl.beta)
    a = WS.image(Gl, h, h, wl.scale, wl.scale, 1.0)
    b = IM.image_conv(G, h, h)
    assert np.max(np.abs(a - b)) <= 1e-12 * np.max(np.abs(b))


def _point_source(L=7, dw=60.0):
    n, beta, S, fov = 128, 8, 7, 0.2
    taps = W.pswf_taps(S, beta)
    rng = np.random.Generator(np.random.PCG64(9))
    nrec = 400
    xc = rng.integers(-40 * beta, 40 * beta, (nrec, 2)) / beta
    w = WS.layer_w(L, dw)[rng.integers(0, L, nrec)]
    u, v = xc[:, 0] / fov, xc[:, 1] / fov
    uvw = np.stack([u, v, w], 1)
    l0, m0 = -0.04, 0.025
    V = np.exp(-2j * np.pi * (u * l0 + v * m0 + w * (np.sqrt(1 - l0 ** 2 - m0 ** 2) - 1)))
    lg = (np.arange(n) - n // 2) / n * fov
    Lg, Mg = np.meshgrid(lg, lg)
    truth = np.tensordot(V, np.exp(2j * np.pi * (
        np.multiply.outer(u, Lg) + np.multiply.outer(v, Mg)
        + np.multiply.outer(w, np.sqrt(1 - Lg ** 2 - Mg ** 2) - 1))), 1)
    return n, beta, S, fov, taps, uvw, V, truth, L, dw


def test_point_source_through_w_stacking():
    n, beta, S, fov, taps, uvw, V, truth, L, dw = _point_source()
    geom = oracle.Geometry(nu=n, nv=n, beta=beta, scale_u=fov, scale_v=fov, support=S)
    Gl, sk = WS.grid_layers(geom, taps, uvw, V[:, None], L, 1 / dw)
    assert sk == 0
    h = IM.corrector(n, beta, taps, beta, nn_sinc=False)
    c = slice(n // 4, 3 * n // 4)

    def err(dw_screen):
        img = WS.image(Gl, h, h, fov, fov, dw_screen)[0]
        return np.linalg.norm((img - truth)[c, c]) / np.linalg.norm(truth[c, c])

    assert err(dw) < 2e-4
    assert err(0.0) > 0.3          # no W-term correction
    assert err(-dw) > 0.3          # g_w instead of gbar_w
