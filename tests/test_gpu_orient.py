"""GPU parity of pft_orientation_average (orientation-averaged intensity) against the FP64 oracle."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle as O
import paper_2104_08309_amd as pft
from gpu_util import TOL_FP32C, TOL_FP64, dev, host, nrel, step

pytestmark = pytest.mark.gpu


def run(v, t, qabs, d, w, mode):
    r = pft.orientation_average(dev(v, torch.float64), dev(t, torch.int32), dev(qabs, torch.float64),
                                dev(d, torch.float64), dev(w, torch.float64), mode=mode)
    torch.cuda.synchronize()
    return host(r)


def test_small_mesh_both_forms(gpu):
    """768 (magnitude, direction) pairs (caller's order), including |Q| = 0 (I = V^2)."""
    rng = np.random.default_rng(31)
    rot = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    v, t = mg.icosphere(2, 1.7)
    v = v @ rot.T + np.array([0.3, -0.6, 0.2])
    qabs = np.array([0.0, 1e-3, 0.5, 1.0, 2.0, 4.0])
    d, w = mg.sphere_quadrature(8, 16)
    want = O.orientation_average(v, t, qabs, d, w)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"orientation average small {mode}")
        got = run(v, t, qabs, d, w, mode)
        assert nrel(got, want) < tol, mode
        assert np.all(np.abs(got - want) <= tol * np.abs(want) + 1e-300), mode


def test_sorted_size_ellipsoid(gpu):
    """40 magnitudes x 512 directions = 20480 pairs: the Morton-ordered path."""
    rng = np.random.default_rng(32)
    v, t = mg.ellipsoid_uv([3.0, 2.0, 1.5], 9, rot=np.linalg.qr(rng.normal(size=(3, 3)))[0], centre=(1.0, 0.5, -1.0))
    qabs = np.linspace(0.0, 3.0, 40)
    d, w = mg.sphere_quadrature(16, 32)
    want = O.orientation_average(v, t, qabs, d, w)
    for mode, tol in (("fp64", TOL_FP64), ("fp32c", TOL_FP32C)):
        step(f"orientation average ellipsoid {mode}")
        got = run(v, t, qabs, d, w, mode)
        e = nrel(got, want)
        print(f"{mode} rel err {e:.3e}")
        assert e < tol, mode


def test_empty_quadrature_and_no_magnitudes(gpu):
    v, t = mg.box()
    step("orientation average: no directions")
    got = run(v, t, np.array([0.5, 1.0]), np.zeros((0, 3)), np.zeros(0), "fp32c")
    assert np.array_equal(got, np.zeros(2))
    step("orientation average: no magnitudes")
    assert run(v, t, np.zeros(0), *mg.sphere_quadrature(2, 4), "fp64").shape == (0,)


def test_config2_mesh_full_size_sampled(gpu):
    """Config 2's mesh with 256 magnitudes in (0, 0.5] x a 32 x 32 direction rule (262144 Q, the size of
    config 2's grid): FP32C against the FP64 form everywhere, both against the oracle at two magnitudes."""
    cfg = mg.config2()
    v, t = cfg["verts"], cfg["tris"]
    qabs = np.linspace(0.5 / 256, 0.5, 256)
    d, w = mg.sphere_quadrature(32, 32)
    step("orientation average config-2 mesh fp64")
    I64 = run(v, t, qabs, d, w, "fp64")
    step("orientation average config-2 mesh fp32c")
    I32 = run(v, t, qabs, d, w, "fp32c")
    assert nrel(I32, I64) < TOL_FP32C
    idx = [17, 203]
    want = O.orientation_average(v, t, qabs[idx], d, w)
    assert nrel(I64[idx], want) < TOL_FP64
    assert nrel(I32[idx], want) < TOL_FP32C
