"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle.

Bar: indices bit-exact; grid and degrid values within relative L2 1e-5
(FP32 arithmetic against the FP64 definition); skipped counts exact.
"""
import ctypes as C
import math

import numpy as np
import pytest

import oracle
from paper_2111_04141_amd import workload as W
from tests import helpers as H

pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def api(torch_cuda):
    from paper_2111_04141_amd import api as A
    A.lib()
    return A


@pytest.fixture(scope="module")
def small_sep():
    return W.config_small()


@pytest.fixture(scope="module")
def small_wproj():
    # all four gridder classes (supports 8 .. 64), several hundred tiles
    return W.config_wproj(n_ant=40, n_times=8, n_chan=16, n=1024, nplanes=16, s_min=8,
                          s_max=64, name="wproj-1024-P16-S8to64")


def _edge_uvw(wl, rng):
    """Ties of the nearest-pixel rule, out-of-grid and non-finite records."""
    n, s = wl.n, wl.scale
    rows = []
    for q in range(-40, 40, 7):
        x = (q + 0.5) / wl.beta + 3.0       # beta*x + 1/2 integral
        rows.append([x / s, -x / s, 0.0])
    rows += [[n / s, 0, 0], [-n / (2 * s), 0, 0], [(n / 2 - 1) / s, 0, 0],
             [np.nan, 0, 0], [0, np.inf, 0], [0, 0, np.nan]]
    return np.array(rows, np.float64)


def _to_dev(torch, a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.mark.parametrize("which,uvw_dtype", [("sep", "f32"), ("sep", "f64"),
                                             ("wproj", "f32"), ("wproj", "f64")])
def test_indices_bit_exact(torch_cuda, api, small_sep, small_wproj, which, uvw_dtype):
    torch = torch_cuda
    wl = small_sep if which == "sep" else small_wproj
    rng = np.random.Generator(np.random.PCG64(1))
    uvw = np.concatenate([wl.uvw.astype(np.float64), _edge_uvw(wl, rng)])
    if uvw_dtype == "f32":
        uvw = uvw.astype(np.float32)
    ref = oracle.index(H.oracle_geom(wl), uvw)
    got = api.compute_indices(H.grid_spec(wl), H.device_bank(wl), _to_dev(torch, uvw))
    torch.cuda.synchronize()
    valid = got["valid"].cpu().numpy()
    assert np.array_equal(valid, ref["valid"])
    v = valid.astype(bool)
    for k in ("k_lo_u", "k_lo_v", "o_u", "o_v"):
        assert np.array_equal(got[k].cpu().numpy()[v], ref[k][v]), k
    fin = np.all(np.isfinite(uvw), axis=1)
    assert np.array_equal(got["plane"].cpu().numpy()[fin], ref["plane"][fin])
    assert int(got["nskipped"].item()) == ref["nskipped"]
    assert ref["nskipped"] >= 5


def _grid_both(torch, api, wl, vis, npol=4, dtype="f32", uvw=None):
    uvw = wl.uvw if uvw is None else uvw
    G_ref, sk = oracle.grid(H.oracle_geom(wl), H.oracle_taps(wl, dtype), uvw, vis[:, :npol])
    spec = H.grid_spec(wl, npol)
    nsk = torch.zeros(1, dtype=torch.int64, device="cuda")
    G = api.grid(spec, H.device_bank(wl, dtype), _to_dev(torch, uvw),
                 _to_dev(torch, vis[:, :npol].astype(np.complex64)), nskipped=nsk)
    torch.cuda.synchronize()
    assert int(nsk.item()) == sk
    return G.cpu().numpy(), G_ref


@pytest.mark.parametrize("npol", [4, 1, 2, 3])
def test_grid_separable_small_config(torch_cuda, api, small_sep, npol):
    vis = W.vis_normal(small_sep.nrec, 4)
    G, G_ref = _grid_both(torch_cuda, api, small_sep, vis, npol)
    for p in range(npol):
        assert H.rel_l2(G[p], G_ref[p]) < TOL, p


def test_grid_wproj_all_classes(torch_cuda, api, small_wproj):
    wl = small_wproj
    ix = oracle.index(H.oracle_geom(wl), wl.uvw)
    S = wl.bank.supports[ix["plane"][ix["valid"] == 1]]
    assert (S <= 8).any() and ((S > 8) & (S <= 16)).any()
    assert ((S > 16) & (S <= 32)).any() and (S > 32).any()
    vis = W.vis_normal(wl.nrec, 4, seed=7)
    G, G_ref = _grid_both(torch_cuda, api, wl, vis)
    assert H.rel_l2(G, G_ref) < TOL


def test_nonfinite_visibilities_follow_the_definition(torch_cuda, api, small_wproj):
    """A NaN or Inf visibility makes exactly the cells of its footprint
    non-finite, as in the definition (the gridders switch to FP32 commits for
    such calls); every other cell keeps its value.  One non-finite record per
    support class."""
    wl = small_wproj
    ix = oracle.index(H.oracle_geom(wl), wl.uvw)
    S = np.where(ix["valid"] == 1, wl.bank.supports[np.maximum(ix["plane"], 0)], 0)
    vis = W.vis_normal(wl.nrec, 4, seed=11).astype(np.complex128)
    picks = []
    for lo, hi in ((1, 8), (9, 16), (17, 32), (33, 64)):
        cand = np.nonzero((S >= lo) & (S <= hi))[0]
        picks.append(int(cand[len(cand) // 2]))
    vis[picks[0], 0] = np.nan
    vis[picks[1], 2] = complex(np.inf, 0.0)
    vis[picks[2], 1] = complex(0.0, np.nan)
    vis[picks[3], 3] = complex(-np.inf, 0.0)
    G, G_ref = _grid_both(torch_cuda, api, wl, vis)
    assert np.isnan(G_ref).any() and np.isinf(G_ref.real).any()
    for part in ("real", "imag"):
        g, r = getattr(G, part), getattr(G_ref, part)
        assert np.array_equal(np.isnan(g), np.isnan(r)), part
        assert np.array_equal(np.isposinf(g), np.isposinf(r)), part
        assert np.array_equal(np.isneginf(g), np.isneginf(r)), part
    fin = np.isfinite(G_ref)
    assert H.rel_l2(G[fin], G_ref[fin]) < TOL


@pytest.mark.parametrize("which", ["sep", "wproj"])
def test_degrid(torch_cuda, api, small_sep, small_wproj, which):
    torch = torch_cuda
    wl = small_sep if which == "sep" else small_wproj
    rng = np.random.Generator(np.random.PCG64(3))
    Gin = (rng.standard_normal((4, wl.n, wl.n)) + 1j * rng.standard_normal((4, wl.n, wl.n))
           ).astype(np.complex64)
    V_ref, sk = oracle.degrid(H.oracle_geom(wl), H.oracle_taps(wl), wl.uvw, Gin)
    V = api.degrid(H.grid_spec(wl), H.device_bank(wl), _to_dev(torch, wl.uvw),
                   _to_dev(torch, Gin)).cpu().numpy()
    assert H.rel_l2(V, V_ref) < TOL
    # every record's 4 values, not only the total
    err = np.abs(V - V_ref).max(axis=1) / (np.abs(V_ref).max(axis=1) + 1e-30)
    assert np.quantile(err, 0.999) < 1e-4


def test_adjoint_on_gpu(torch_cuda, api, small_wproj):
    torch = torch_cuda
    wl = small_wproj
    rng = np.random.Generator(np.random.PCG64(4))
    x = (rng.standard_normal((wl.nrec, 4)) + 1j * rng.standard_normal((wl.nrec, 4))).astype(
        np.complex64)
    y = (rng.standard_normal((4, wl.n, wl.n)) + 1j * rng.standard_normal((4, wl.n, wl.n))).astype(
        np.complex64)
    spec, bank = H.grid_spec(wl), H.device_bank(wl)
    plan = api.Plan(spec, bank, _to_dev(torch, wl.uvw))
    Gx = plan.grid(_to_dev(torch, x)).cpu().numpy().astype(np.complex128)
    Hy = plan.degrid(_to_dev(torch, y)).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(y.astype(np.complex128), Gx)
    rhs = np.vdot(Hy, x.astype(np.complex128))
    assert abs(lhs - rhs) / abs(lhs) < TOL
    plan.close()


def test_plan_reuse_matches_one_shot(torch_cuda, api, small_sep):
    torch = torch_cuda
    wl = small_sep
    vis = _to_dev(torch, W.vis_normal(wl.nrec, 4, seed=9))
    uvw = _to_dev(torch, wl.uvw)
    spec, bank = H.grid_spec(wl), H.device_bank(wl)
    one = api.grid(spec, bank, uvw, vis)
    with api.Plan(spec, bank, uvw) as plan:
        g = plan.grid(vis)
        plan.grid(vis, out=g)                      # accumulates
        assert plan.nskipped == 0
        assert plan.nbytes > 0
        d1 = plan.degrid(one)
    d0 = api.degrid(spec, bank, uvw, one)
    torch.cuda.synchronize()
    assert H.rel_l2(g.cpu().numpy(), 2 * one.cpu().numpy()) < TOL
    assert H.rel_l2(d1.cpu().numpy(), d0.cpu().numpy()) < TOL


def test_empty_and_all_skipped(torch_cuda, api, small_sep):
    torch = torch_cuda
    wl = small_sep
    spec, bank = H.grid_spec(wl), H.device_bank(wl)
    uvw0 = torch.zeros(0, 3, device="cuda")
    vis0 = torch.zeros(0, 4, dtype=torch.complex64, device="cuda")
    g = api.grid(spec, bank, uvw0, vis0)
    assert float(g.abs().max()) == 0.0
    assert api.degrid(spec, bank, uvw0, g).shape == (0, 4)
    far = torch.full((1000, 3), 1e9, device="cuda")
    vis = torch.ones(1000, 4, dtype=torch.complex64, device="cuda")
    nsk = torch.zeros(1, dtype=torch.int64, device="cuda")
    g = api.grid(spec, bank, far, vis, nskipped=nsk)
    assert int(nsk.item()) == 1000 and float(g.abs().max()) == 0.0
    v = api.degrid(spec, bank, far, torch.ones_like(g))
    assert float(v.abs().max()) == 0.0


def test_single_record_and_hot_cell(torch_cuda, api, small_sep, small_wproj):
    """One record; and 200k records on one NN pixel (the thesis's
    Maximum Performance input, Section 3.4.4), the worst case for
    same-cell contention."""
    torch = torch_cuda
    for wl in (small_sep, small_wproj):
        one = np.array([[3.3 / wl.scale, -7.7 / wl.scale, 0.1]])
        vis = W.vis_normal(1, 4, seed=5)
        G, G_ref = _grid_both(torch, api, wl, vis, uvw=one)
        assert H.rel_l2(G, G_ref) < TOL
        hot = np.repeat(np.array([[12.26 / wl.scale, 30.1 / wl.scale, 0.0]]), 200_000, axis=0)
        vis = W.vis_normal(hot.shape[0], 4, seed=6)
        G, G_ref = _grid_both(torch, api, wl, vis, uvw=hot)
        assert H.rel_l2(G, G_ref) < TOL


def test_large_finite_visibilities_commit_in_fp32(torch_cuda, api, small_sep, small_wproj):
    """64 records on one pixel with visibilities near 1e36: the window
    gridders' fixed-point bound (2 max|tap| times the sum of the records'
    largest components) overflows FP32 although every cell sum is far below
    it; such units must commit in FP32 instead (the result stays finite and
    matches the definition)."""
    torch = torch_cuda
    for wl in (small_sep, small_wproj):
        hot = np.repeat(np.array([[20.3 / wl.scale, -11.6 / wl.scale, 0.0]]), 64, axis=0)
        vis = W.vis_normal(hot.shape[0], 4, seed=8) * 2e36
        G, G_ref = _grid_both(torch, api, wl, vis, uvw=hot)
        assert np.isfinite(G).all() and np.isfinite(G_ref).all()
        assert H.rel_l2(G, G_ref) < TOL


@pytest.mark.parametrize("dtype", ["f16", "bf16"])
def test_reduced_precision_bank(torch_cuda, api, small_wproj, dtype):
    """FP16/BF16 taps, FP32 arithmetic.  Against the oracle run on the same
    quantised taps the error is accumulation only (bar 1e-5); against the
    full-precision bank the total error is bounded by the format's unit
    roundoff (2^-11 for FP16, 2^-8 for BF16) times a small factor."""
    wl = small_wproj
    vis = W.vis_normal(wl.nrec, 4, seed=8)
    G, G_q = _grid_both(torch_cuda, api, wl, vis, dtype=dtype)
    assert H.rel_l2(G, G_q) < TOL
    G_full, _ = oracle.grid(H.oracle_geom(wl), wl.bank.taps, wl.uvw, vis)
    u = 2.0 ** -11 if dtype == "f16" else 2.0 ** -8
    err = H.rel_l2(G, G_full)
    assert err < 2 * u, err


def test_plan_in_torch_workspace_and_library_owned(torch_cuda, api, small_sep):
    """A plan's device arrays live in the workspace the binding allocates
    with torch (torch's allocator accounts for them); a plan created through
    the C ABI without a workspace owns a stream-ordered arena, which
    mg_plan_destroy releases after the plan's last calls, here queued on two
    streams just before the destroy."""
    torch = torch_cuda
    wl = small_sep
    spec, bank = H.grid_spec(wl), H.device_bank(wl)
    uvw = _to_dev(torch, wl.uvw)
    vis = _to_dev(torch, W.vis_normal(wl.nrec, 4, seed=14))
    need = api.workspace_size(spec, bank, wl.nrec)
    torch.cuda.synchronize()
    before = torch.cuda.memory_allocated()
    plan = api.Plan(spec, bank, uvw)
    assert torch.cuda.memory_allocated() - before >= need
    assert plan.nbytes == need
    g1 = plan.grid(vis)
    L = api.lib()
    h = C.c_void_p()
    gd, kd = spec.desc(), bank.desc()
    cur = torch.cuda.current_stream()
    assert L.mg_plan_create(C.byref(h), C.byref(gd), C.byref(kd), wl.nrec, uvw.data_ptr(),
                            api.MG_F64, None, cur.cuda_stream) == api.MG_OK
    g2 = torch.zeros_like(g1)
    assert L.mg_plan_grid(h, vis.data_ptr(), g2.data_ptr(), cur.cuda_stream) == api.MG_OK
    side = torch.cuda.Stream()
    side.wait_stream(cur)
    v2 = torch.empty_like(vis)
    assert L.mg_plan_degrid(h, g1.data_ptr(), v2.data_ptr(), side.cuda_stream) == api.MG_OK
    assert L.mg_plan_destroy(h) == api.MG_OK
    torch.cuda.synchronize()
    v1 = plan.degrid(g1)
    torch.cuda.synchronize()
    assert H.rel_l2(g2.cpu().numpy(), g1.cpu().numpy()) < 1e-6
    assert H.rel_l2(v2.cpu().numpy(), v1.cpu().numpy()) < 1e-6
    G_ref, _ = oracle.grid(H.oracle_geom(wl), H.oracle_taps(wl), wl.uvw, vis.cpu().numpy())
    assert H.rel_l2(g1.cpu().numpy(), G_ref) < TOL
    held = torch.cuda.memory_allocated()
    plan.close()
    torch.cuda.synchronize()
    assert held - torch.cuda.memory_allocated() >= need
