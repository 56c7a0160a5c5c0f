"""GPU parity of pft_intensity_loss_3d (fused forward, intensity-loss cotangent and adjoint) against the
FP64 oracle and against the unfused path through the same library."""
import numpy as np
import pytest
import torch

import meshgen as mg
import oracle as O
import paper_2104_08309_amd as pft
from gpu_util import dev, host, nrel, step

pytestmark = pytest.mark.gpu


def loss_case(level=3, n=32, seed=2):
    """Perturbed icosphere against the intensity of the unperturbed one (the adjoint's workload, small)."""
    v0, t = mg.icosphere(level, 5.0)
    rng = np.random.default_rng(seed)
    v = mg.perturb_radial(v0, 0.02, rng)
    q = mg.q_slice_z(n, 0.8)
    target = np.abs(O.ft3d(v0, t, q)) ** 2
    w = rng.uniform(0.5, 1.5, size=len(q)) / (len(q) * O.volume3d(v0, t) ** 4)
    return v, t, q, target, w


def oracle_loss(v, t, q, target, w):
    F = O.ft3d(v, t, q)
    r = np.abs(F) ** 2 - target
    return float(np.sum(w * r * r)), O.grad3d(v, t, q, 4 * w * r * F), F


def run(v, t, q, target, w, mode, **kw):
    return pft.intensity_loss_3d(dev(v), dev(t, torch.int32), dev(q), dev(target),
                                 None if w is None else dev(w), mode=mode, **kw)


# The loss amplifies the error of F: with r = |F|^2 - I about 4 % of |F|^2 for a 2 % perturbation,
# a relative error e in F gives about 2 e |F|^2 / |r| = 50 e in r. The FP32C bars below are the
# transform's 1e-5 bar times that factor, rounded up (the FP64 bars stay tight).
def test_loss_and_gradient_against_oracle(gpu):
    v, t, q, target, w = loss_case()
    L, G, F = oracle_loss(v, t, q, target, w)
    for mode, tol_l, tol_g in (("fp64", 1e-11, 1e-9), ("fp32c", 1e-4, 1e-4)):
        step(f"fused loss {mode}")
        loss, gv, Fg = run(v, t, q, target, w, mode, return_F=True)
        torch.cuda.synchronize()
        assert abs(loss.item() - L) < tol_l * L, mode
        e = nrel(host(gv), G)
        print(f"fused loss {mode}: grad rel err {e:.3e}")
        assert e < tol_g, mode
        assert nrel(host(Fg), F) < (1e-12 if mode == "fp64" else 1e-5), mode
        # |F|^2 is translation invariant: the vertex gradients sum to zero
        assert np.max(np.abs(host(gv).sum(axis=0))) < 1e-3 * np.max(np.abs(host(gv)))


def test_matches_unfused_path_and_unit_weights(gpu):
    """forward_3d, the loss in torch and backward_3d give the same loss and gradient; w = None is w = 1."""
    v, t, q, target, w = loss_case(level=2, n=24, seed=3)
    V, T, Q = dev(v), dev(t, torch.int32), dev(q)
    for mode in ("fp64", "fp32c"):
        step(f"fused vs unfused {mode}")
        F = pft.forward_3d(V, T, Q, mode=mode).to(torch.complex128)
        r = F.real ** 2 + F.imag ** 2 - dev(target)
        L_ref = torch.sum(r * r).item()
        g = 4 * r * F
        cdt = torch.complex128 if mode == "fp64" else torch.complex64
        G_ref = host(pft.backward_3d(V, T, Q, g.to(cdt), mode=mode))
        loss, gv = run(v, t, q, target, None, mode)
        torch.cuda.synchronize()
        # FP32C: the unfused path rounds F to complex64 before the loss (see the factor above)
        tol = 1e-12 if mode == "fp64" else 1e-4
        assert abs(loss.item() - L_ref) <= tol * abs(L_ref), mode
        assert nrel(host(gv), G_ref) < tol, mode


def test_autograd_and_loss_only(gpu):
    v, t, q, target, w = loss_case(level=2, n=24, seed=4)
    step("fused loss through autograd")
    V = dev(v).requires_grad_(True)
    loss = pft.fused_intensity_loss(V, dev(t, torch.int32), dev(q), dev(target), dev(w), mode="fp64")
    (3.0 * loss).backward()
    torch.cuda.synchronize()
    L, G, _ = oracle_loss(v, t, q, target, w)
    assert abs(loss.item() - L) < 1e-11 * L
    assert nrel(host(V.grad), 3.0 * G) < 1e-9
    step("fused loss without gradient; empty Q list")
    loss2, gv2 = run(v, t, q, target, w, "fp32c", need_grad=False)
    assert gv2 is None and abs(loss2.item() - L) < 1e-4 * L
    z = torch.zeros((0, 3), dtype=torch.float64, device="cuda:0")
    e = torch.zeros(0, dtype=torch.float64, device="cuda:0")
    loss3, gv3 = pft.intensity_loss_3d(dev(v), dev(t, torch.int32), z, e, None, mode="fp32c")
    torch.cuda.synchronize()
    assert loss3.item() == 0.0 and torch.count_nonzero(gv3).item() == 0


def test_config4_full_size(gpu):
    """Config 4 (81920 faces x 65536 Q, the adjoint workload). The loss weights every Q alike, so the
    gradient carries the forward's error amplified by the loss; to test the fused FP32C adjoint itself,
    its gradient is compared with the FP64 adjoint applied to the cotangent formed from the FP32C
    forward (both then share that amplified error). Also: FP32C against FP64 loss, and the
    translation identity sum_k dL/dv_k = 0 at full size."""
    cfg = mg.config4()
    v, t, q = cfg["verts"], cfg["tris"], cfg["q"]
    V, T, Q = dev(v), dev(t, torch.int32), dev(q)
    step("config 4 target (fp64 forward of the unperturbed sphere)")
    target = host(pft.forward_3d(dev(cfg["verts0"]), T, Q, mode="fp64", intensity=True)[1])
    w = np.full(len(q), 1.0 / (len(q) * (4.0 / 3.0 * np.pi * 50.0 ** 3) ** 4))
    step("config 4 fused loss fp32c")
    L32, G32, F32 = run(v, t, q, target, w, "fp32c", return_F=True)
    step("config 4 fp64 adjoint of the fp32c cotangent")
    F32 = host(F32).astype(np.complex128)
    r = np.abs(F32) ** 2 - target
    Gref = host(pft.backward_3d(V, T, Q, dev(4 * w * r * F32), mode="fp64"))
    G32 = host(G32).astype(np.float64)
    e = nrel(G32, Gref)
    print(f"config 4 fused fp32c adjoint vs fp64 adjoint of the same cotangent: {e:.3e}")
    # The intensity-loss gradient is a small residual of large per-Q contributions (|F|^2 is
    # translation invariant, so they cancel in sum over the vertices), which raises the relative
    # error of the binary32 adjoint from its 1e-7 level with generic cotangents to about 3e-5 here;
    # the cotangent of the reference is also formed from F rounded to complex64.
    assert e < 1e-4
    step("config 4 fused loss fp64")
    L64, G64 = run(v, t, q, target, w, "fp64")
    torch.cuda.synchronize()
    assert abs(L32.item() - L64.item()) < 1e-4 * L64.item()
    G64 = host(G64)
    for G, tol in ((G64, 1e-8), (G32, 1e-4)):
        assert np.max(np.abs(G.sum(axis=0))) < tol * np.max(np.abs(G)) * np.sqrt(len(v))


def test_f32_inputs(gpu):
    """float32 vertices and Q: the fused loss's gradient is float32 and matches the unfused path."""
    v, t, q, target, w = loss_case(level=2, n=24, seed=5)
    V, T, Q = dev(v, torch.float32), dev(t, torch.int32), dev(q, torch.float32)
    step("fused loss f32 inputs")
    loss, gv = pft.intensity_loss_3d(V, T, Q, dev(target), dev(w), mode="fp32c")
    F = pft.forward_3d(V, T, Q, mode="fp32c").to(torch.complex128)
    r = F.real ** 2 + F.imag ** 2 - dev(target)
    G_ref = host(pft.backward_3d(V, T, Q, (4 * dev(w) * r * F).to(torch.complex64), mode="fp32c"))
    torch.cuda.synchronize()
    assert gv.dtype == torch.float32
    L_ref = torch.sum(dev(w) * r * r).item()
    assert abs(loss.item() - L_ref) <= 1e-4 * abs(L_ref)
    assert nrel(host(gv), G_ref) < 1e-4
