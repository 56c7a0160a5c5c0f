"""Bitwise reproducibility of the entry points: two calls on the same inputs give identical bytes
(fixed reduction orders, no floating-point atomics), at sizes that take the Morton-ordered path."""
import numpy as np
import pytest
import torch

import meshgen as mg
import paper_2104_08309_amd as pft
from gpu_util import dev, host, step

pytestmark = pytest.mark.gpu


def same(a, b):
    if isinstance(a, (tuple, list)):
        return all(same(x, y) for x, y in zip(a, b))
    if a is None:
        return b is None
    x, y = np.atleast_1d(host(a)), np.atleast_1d(host(b))
    return x.shape == y.shape and np.array_equal(x.view(np.uint8), y.view(np.uint8))


def twice(fn):
    a = fn()
    torch.cuda.synchronize()
    b = fn()
    torch.cuda.synchronize()
    return a, b


def test_regions_loss_poly_orientation_and_batch_repeat(gpu):
    rng = np.random.default_rng(61)
    v, t, off = mg.layered_sphere(2, [0.6, 0.9, 1.2])
    V, T = dev(v, torch.float32), dev(t, torch.int32)
    Q = dev(mg.q_random_ball(10000, 10.0, rng), torch.float32)
    rho = dev(np.array([1.0, -0.5, 2.0]))
    g = torch.randn(Q.shape[0], dtype=torch.complex64, device="cuda:0",
                    generator=torch.Generator(device="cuda:0").manual_seed(1))
    for mode in ("fp32c", "fp64"):
        VV, QQ = (V.double(), Q.double()) if mode == "fp64" else (V, Q)
        gg = g.to(torch.complex128) if mode == "fp64" else g
        step(f"repeat regions forward {mode}")
        a, b = twice(lambda: pft.forward_3d_regions(VV, T, off, rho, QQ, mode=mode, per_region=True))
        assert same(a, b), mode
        step(f"repeat regions backward {mode}")
        a, b = twice(lambda: pft.backward_3d_regions(VV, T, off, rho, QQ, gg, mode=mode))
        assert same(a, b), mode
        step(f"repeat intensity loss {mode}")
        target = torch.rand(Q.shape[0], dtype=torch.float64, device="cuda:0",
                            generator=torch.Generator(device="cuda:0").manual_seed(2))
        a, b = twice(lambda: pft.intensity_loss_3d(VV, T, QQ, target, None, mode=mode))
        assert same(a, b), mode
    step("repeat polygon faces")
    pv, pf = mg.ellipsoid_quads([2.0, 1.5, 1.0], 10, 16)
    a, b = twice(lambda: pft.forward_3d_poly(dev(pv, torch.float32), pf, Q, mode="fp32c"))
    assert same(a, b)
    step("repeat orientation average")
    d, w = mg.sphere_quadrature(12, 24)
    qa = dev(np.linspace(0.0, 5.0, 40))
    a, b = twice(lambda: pft.orientation_average(V.double(), T, qa, dev(d), dev(w), mode="fp32c"))
    assert same(a, b)
    step("repeat batch")
    meshes = [{"verts": mg.icosphere(2, 1.0 + 0.3 * i)[0], "tris": mg.icosphere(2, 1.0)[1],
               "q": mg.q_random_ball(3000 + 500 * i, 6.0, rng)} for i in range(4)]
    vo, to, qo = [0], [0], [0]
    for m in meshes:
        vo.append(vo[-1] + len(m["verts"]))
        to.append(to[-1] + len(m["tris"]))
        qo.append(qo[-1] + len(m["q"]))
    BV = dev(np.concatenate([m["verts"] for m in meshes]), torch.float32)
    BT = dev(np.concatenate([m["tris"] for m in meshes]), torch.int32)
    BQ = dev(np.concatenate([m["q"] for m in meshes]), torch.float32)
    BG = torch.randn(qo[-1], dtype=torch.complex64, device="cuda:0",
                     generator=torch.Generator(device="cuda:0").manual_seed(3))
    a, b = twice(lambda: (pft.batch_forward(BV, BT, BQ, vo, to, qo, mode="fp32c"),
                          pft.batch_backward(BV, BT, BQ, vo, to, qo, BG, mode="fp32c")))
    assert same(a, b)


def test_workspace_streams_threads_and_release(gpu):
    """Temporaries live in a per-stream workspace: calls on two streams from two host threads at once,
    and calls after pft_release_workspace, give the same bytes as a plain call."""
    import threading
    rng = np.random.default_rng(62)
    v, t = mg.icosphere(3, 1.3)
    V, T = dev(v, torch.float32), dev(t, torch.int32)
    Qs = [dev(mg.q_random_ball(9000 + 1000 * i, 6.0, rng), torch.float32) for i in range(2)]
    step("workspace: reference calls")
    ref = [host(pft.forward_3d(V, T, Q, mode="fp32c")) for Q in Qs]
    streams = [torch.cuda.Stream() for _ in range(2)]
    got = [None, None]

    def work(i):
        with torch.cuda.stream(streams[i]):
            for _ in range(3):
                F = pft.forward_3d(V, T, Qs[i], mode="fp32c")
            streams[i].synchronize()
            got[i] = host(F)

    step("workspace: two streams from two threads")
    th = [threading.Thread(target=work, args=(i,)) for i in range(2)]
    for x in th:
        x.start()
    for x in th:
        x.join()
    for i in range(2):
        assert np.array_equal(got[i].view(np.uint8), ref[i].view(np.uint8))
    step("workspace: release and call again")
    pft.release_workspace()
    again = host(pft.forward_3d(V, T, Qs[0], mode="fp32c"))
    assert np.array_equal(again.view(np.uint8), ref[0].view(np.uint8))
