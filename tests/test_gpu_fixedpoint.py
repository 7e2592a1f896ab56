"""The window gridders' fixed-point commits on coherent inputs, where
rounding errors of one sign would add up: every visibility 1 (the point
spread function input of the thesis's validation, Section 8.1.2), a single
point source, and visibilities with bright outliers.  Against the FP64
oracle at relative L2 1e-5 over the grid, and cell by cell against the bound
the commits and FP32 sums allow (tests/helpers.py fixed_point_cell_bound)."""
import numpy as np
import pytest

import oracle
from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def api():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_04141_amd import api as A
    A.lib()
    return A


@pytest.fixture(scope="module")
def small_sep():
    return W.config_small()


@pytest.fixture(scope="module")
def small_wproj():
    return W.config_wproj(n_ant=40, n_times=8, n_chan=16, n=1024, nplanes=16, s_min=8,
                          s_max=64, name="wproj-1024-P16-S8to64")


def _inputs(wl, kind, rng):
    n = wl.nrec
    if kind == "psf":
        return np.ones((n, 4), np.complex128)
    if kind == "point":
        # one point source at (l0, m0) rad: V = A exp(-j2pi (u l0 + v m0))
        l0, m0 = 0.37 / wl.scale, -0.21 / wl.scale
        ph = np.exp(-2j * np.pi * (wl.uvw[:, 0].astype(np.float64) * l0 +
                                   wl.uvw[:, 1].astype(np.float64) * m0))
        return ph[:, None] * np.array([1.0, 0.5, 0.25j, -1.0])[None, :]
    v = (rng.standard_normal((n, 4)) + 1j * rng.standard_normal((n, 4)))
    v[::97] *= 1e4            # bright outliers, about one in 97 records
    return v


def _grid(api, wl, vis):
    import torch
    G = api.grid(H.grid_spec(wl), H.device_bank(wl), torch.from_numpy(wl.uvw).cuda(),
                 torch.from_numpy(vis.astype(np.complex64)).cuda())
    torch.cuda.synchronize()
    return G.cpu().numpy()


@pytest.mark.parametrize("kind", ["psf", "point", "outliers"])
@pytest.mark.parametrize("which", ["sep", "wproj"])
def test_coherent_inputs_small(api, small_sep, small_wproj, which, kind):
    wl = small_sep if which == "sep" else small_wproj
    rng = np.random.Generator(np.random.PCG64(31))
    vis = _inputs(wl, kind, rng).astype(np.complex64).astype(np.complex128)
    G = _grid(api, wl, vis)
    geom, taps = H.oracle_geom(wl), H.oracle_taps(wl)
    G_ref, _ = oracle.grid(geom, taps, wl.uvw, vis)
    err = H.rel_l2(G, G_ref)
    print(f"[fixedpoint] {which} {kind}: rel-L2 {err:.2e}", flush=True)
    assert err < TOL, err
    bound, n_c = H.fixed_point_cell_bound(geom, taps, wl.uvw, vis, wl.support)
    H.assert_within_cell_bound(G, G_ref, bound, (which, kind))
    if kind == "outliers":
        # cells no outlier can reach keep the accuracy of ordinary inputs
        clean = (bound < 1e-3 * np.abs(G_ref).max()) & (np.abs(G_ref) > 0)
        assert clean.any()
        rel = np.abs(G - G_ref)[clean] / np.abs(G_ref)[clean]
        print(f"[fixedpoint] {which} outliers: {int(clean.sum())} cells away from outliers, "
              f"median rel {np.median(rel):.2e}", flush=True)
