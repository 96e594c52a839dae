"""Parity with the FP64 oracle at the full sizes of the benchmark's other
workloads, in the tile shapes it times them with:

* the cylinder + drop physics on 4096 x 4096 (working set far above the
  last-level cache), FP64 with 64 x 8 tiles and FP32 with 64 x 16 tiles,
  over the first 2 steps (the second carries the explicit-Euler time
  derivatives and the lagged velocity of the first);
* the 1024 x 2048 gas-liquid pool with 64 free particles, FP64, FP32 and
  FP16-dev storage with 64 x 8 tiles, over 3 steps, fields and particle
  state; tiles of 4, 8 and 16 rows give bitwise the same result there;
* the 1024 x 1024 cylinder + drop geometry between bounce-back walls,
  FP64 and FP32, over 3 steps;
* the 4096 x 4096 voxel-solid smoothing (20 Cahn-Hilliard steps);
* the 2048 x 1024 porous channel with 200 obstacles, FP64 and FP32, over
  3 steps, and its recipe on a small ragged grid over 200 steps.

Bars as in the small-size parity tests: FP64 <= 1e-12 relative, FP32 <= 1e-5
relative on phi, u and P, in the 2-norm and the max-norm (tests/parity.py),
FP16-dev within its storage quantisation.  The oracle
runs once per workload (about a minute for the 4096 x 4096 step on 16
threads, 11 GB of host memory, and a minute for the smoothing).
"""
import numpy as np
import pytest

from paper_2311_05097_amd import workloads as W
from parity import BAR, check, errors, fmt, rel

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2311_05097_amd import lbmgls
    lbmgls.lib()
    return lbmgls


@pytest.fixture(scope="module")
def r4096():
    from oracle.oracle import Oracle
    w = W.roofline_grid()
    o = Oracle(w.params, *w.arrays())
    o.step(2)
    out = o.read()
    del o
    return w, out


@pytest.mark.parametrize("storage,tile,tol", [("fp64", 8, 1e-12), ("fp32", 16, 1e-5)])
def test_r4096_full_size(gpu, r4096, storage, tile, tol):
    w, ref = r4096
    d = gpu.Domain(w.params, *w.arrays(), storage=storage, tile=tile)
    d.step(2)
    errs = errors(d.read(), ref)
    print(f"\n4096^2 {storage} 64x{tile} 2 steps (2-norm/max-norm): {fmt(errs)}")
    check(errs, tol)


@pytest.fixture(scope="module")
def c5():
    from oracle.oracle import Oracle
    w = W.pool_with_particles()
    o = Oracle(w.params, *w.arrays(), particles=w.particles)
    o.step(3)
    return w, o.read(), o.particles()


def _c5_run(gpu, w, storage, tile):
    d = gpu.Domain(w.params, *w.arrays(), storage=storage, tile=tile, particles=w.particles)
    d.step(3)
    return d.read(), d.particles()


@pytest.mark.parametrize("storage", ["fp64", "fp32", "fp16dev"])
def test_c5_full_size(gpu, c5, storage):
    w, ref, (os_, oo) = c5
    assert len(w.particles) == 64
    fields, (ds, do) = _c5_run(gpu, w, storage, 8)
    errs = errors(fields, ref)
    perr = float(np.abs(ds - os_).max())
    ferr = float(np.abs(do[:, :3] - oo[:, :3]).max() / np.abs(oo[:, :3]).max())
    print(f"\nC5 {storage} 64x8 3 steps (2-norm/max-norm): {fmt(errs)} state={perr:.2e} force={ferr:.2e}")
    if storage == "fp64":
        check(errs, BAR["fp64"])
        assert perr <= 1e-12 and ferr <= 1e-10
    elif storage == "fp32":
        check(errs, BAR["fp32"])
        assert perr <= 1e-6 and ferr <= 1e-4
    else:
        assert errs["phi"][0] <= 1e-3 and perr <= 1e-4


def test_c5_full_size_tiles_bitwise(gpu, c5):
    w = c5[0]
    runs = [_c5_run(gpu, w, "fp32", t) for t in (4, 8, 16)]
    flat = [list(f) + list(p) for f, p in runs]
    for other in flat[1:]:
        for a, b in zip(flat[0], other):
            assert np.array_equal(a, b)


@pytest.mark.parametrize("storage,tile,tol", [("fp64", 8, 1e-12), ("fp32", 8, 1e-5), ("fp32", 4, 1e-5)])
def test_c2_channel_walls_full_size(gpu, storage, tile, tol):
    """The 1024 x 1024 cylinder + drop geometry closed by bounce-back walls
    below and above (no gravity, mu1 = 0.3, viscosity ratio 50: the walled
    case the benchmark times), 3 steps against the oracle."""
    from oracle.oracle import Oracle
    w = W.cylinder_drop(1024, 128.0, 160.0, g=0.0)
    w.params.update(mu1=0.3, mu2=0.3 / 50, bounce_y=1)
    o = Oracle(w.params, *w.arrays())
    o.step(3)
    d = gpu.Domain(w.params, *w.arrays(), storage=storage, tile=tile)
    d.step(3)
    errs = errors(d.read(), o.read())
    print(f"\nC2 channel {storage} 64x{tile} 3 steps (2-norm/max-norm): {fmt(errs)}")
    check(errs, tol)


def test_voxel_smoothing_full_size(gpu):
    """The 4096 x 4096 voxel solid of 3000 grains smoothed by 20
    Cahn-Hilliard steps, as timed by the benchmark, against the oracle."""
    from oracle import oracle as O
    s = W.voxel_solid(4096, 4096, n_grains=3000, seed=9, r_range=(6.0, 30.0))
    p = W.params(4096, 4096)
    g = gpu.smooth_solid(p, s, 20)
    o = O.smooth_solid(s, p["D"], 20)
    err = float(np.abs(g - o).max())
    print(f"\nvoxel smoothing 4096^2: max abs diff {err:.2e}")
    assert err <= 1e-13


@pytest.fixture(scope="module")
def c3():
    from oracle.oracle import Oracle
    w = W.config3()
    o = Oracle(w.params, *w.arrays())
    o.step(3)
    return w, o.read()


@pytest.mark.parametrize("storage,tile,tol", [("fp64", 8, 1e-12), ("fp32", 8, 1e-5), ("fp32", 16, 1e-5)])
def test_c3_porous_channel_full_size(gpu, c3, storage, tile, tol):
    """The 2048 x 1024 porous channel (diffuse channel walls, 200 obstacles
    with their own contact angles, density ratio 1000, body force along x),
    3 steps against the oracle."""
    w, ref = c3
    assert len(w.meta["circles"]) == 200
    d = gpu.Domain(w.params, *w.arrays(), storage=storage, tile=tile)
    d.step(3)
    errs = errors(d.read(), ref)
    print(f"\nC3 {storage} 64x{tile} 3 steps (2-norm/max-norm): {fmt(errs)}")
    check(errs, tol)


def test_c3_shaped_small_channel_fp64_200_steps(gpu):
    """The porous-channel recipe on 333 x 150 (ragged in both directions,
    12 obstacles, density ratio 10 so that it stays finite), 200 steps."""
    from oracle.oracle import Oracle
    w = W.porous_channel(nx=333, ny=150, n_obstacles=12, seed=6, r_range=(6.0, 14.0), rho_ratio=10.0,
                         mu_ratio=1.0)
    o = Oracle(w.params, *w.arrays())
    o.step(200)
    d = gpu.Domain(w.params, *w.arrays(), storage="fp64", tile=8)
    d.step(200)
    errs = errors(d.read(), o.read())
    print(f"\nsmall channel fp64 200 steps (2-norm/max-norm): {fmt(errs)}")
    check(errs, BAR["fp64"])


@pytest.mark.parametrize("storage", ["fp16dev", "fp32"])
def test_large_domain_is_the_small_one_tiled(gpu, storage):
    """A periodic 16384 x 16384 domain (2^28 nodes: every population plane
    and offset past 4 GiB) started from the 1024 x 1024 cylinder + drop state
    repeated 16 x 16 times is the 1024 x 1024 problem: after 5 steps its
    fields are that problem's fields repeated, bit for bit, and in the 16-bit
    mode its exact phase mass is 256 times the small domain's."""
    import gc
    w = W.cylinder_drop(1024, 128.0, 160.0, g=0.0)
    w.params.update(mu1=0.3, mu2=0.3 / 50)
    small = gpu.Domain(w.params, *w.arrays(), storage=storage, tile=8)
    small.step(5)
    ref = small.read()
    m_small = small.mass()
    small.close()
    k = 16
    pl = dict(w.params, nx=1024 * k, ny=1024 * k)
    big = gpu.Domain(pl, *[np.tile(a, (k, k)) for a in w.arrays()], storage=storage, tile=8)
    gc.collect()
    big.step(5)
    m_big = big.mass()
    got = big.read()
    big.close()
    for a, b in zip(got, ref):
        assert a.shape == (1024 * k, 1024 * k)
        assert np.array_equal(a.reshape(k, 1024, k, 1024), np.broadcast_to(b[None, :, None, :], (k, 1024, k, 1024)))
    if storage == "fp16dev":
        assert m_big == 256.0 * m_small
    else:
        assert abs(m_big - 256.0 * m_small) <= 1e-9 * abs(256.0 * m_small) + 1e-6
