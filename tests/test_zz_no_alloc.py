"""pft_forward_3d_noalloc (temporaries in a fixed device array, no allocation in the call) against
pft_forward_3d on the same inputs: two calls in a row, the second smaller, in both forms; and the
size limit of the array."""
import numpy as np
import pytest
import torch

import meshgen as mg
import paper_2104_08309_amd as pft
from gpu_util import TOL_FP32C, TOL_FP64, dev, host, nrel, step
from paper_2104_08309_amd._lib import PFT_EINVAL, PftError

pytestmark = pytest.mark.gpu


def test_noalloc_matches_forward_3d_two_calls(gpu):
    rng = np.random.default_rng(21)
    v1, t1 = mg.icosphere(3, 4.0)
    v1 = v1 + np.array([0.7, -0.4, 1.1])
    q1 = np.concatenate([[[0.0, 0.0, 0.0]], mg.q_random_ball(20000, 3.0, rng)])
    v2, t2 = mg.ellipsoid_uv([2.0, 1.5, 1.0], 9, centre=(0.3, 0.2, -0.5))
    q2 = np.concatenate([[[0.0, 0.0, 1e-4]], mg.q_random_ball(3000, 5.0, rng)])
    for mode, tol in (("fp32c", TOL_FP32C), ("fp64", TOL_FP64)):
        for i, (v, t, q) in enumerate(((v1, t1, q1), (v2, t2, q2))):
            V, T, Q = dev(v), dev(t, torch.int32), dev(q)
            step(f"noalloc call {i} ({t.shape[0]} faces x {q.shape[0]} Q) {mode}")
            F, I = pft.forward_3d_noalloc(V, T, Q, mode=mode, intensity=True)
            step(f"forward_3d reference call {i} {mode}")
            Fr, Ir = pft.forward_3d(V, T, Q, mode=mode, intensity=True)
            torch.cuda.synchronize()
            e = nrel(host(F), host(Fr))
            print(f"noalloc {mode} call {i}: rel diff {e:.2e}")
            assert e < tol
            assert nrel(host(I), host(Ir)) < 2 * tol


def test_noalloc_size_limit(gpu):
    """A Q list whose partial sums cannot fit beside the records is refused before any GPU work."""
    v, t = mg.icosphere(1, 1.0)
    V, T = dev(v), dev(t, torch.int32)
    q = torch.zeros((5_000_000, 3), dtype=torch.float32, device="cuda:0")
    step("noalloc oversize Q list")
    with pytest.raises(PftError) as ei:
        pft.forward_3d_noalloc(V, T, q, mode="fp32c")
    assert ei.value.status == PFT_EINVAL and "too many Q" in str(ei.value)
