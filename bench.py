"""Throughput of the direct polyhedron Fourier transform on one MI355X.

Workload (default): closed icosphere mesh, subdivision level 4 (5120
triangles, 2562 vertices), radius 50, with Q on the 64^3 FFT-style grid over
[-0.5, 0.5)^3 (262144 Q, containing Q = 0, the axes and the (1,1,1) diagonal).
One step = the whole hot path on that input: pft_forward_3d (per-face records,
Q staging, per-(Q, face) edge sums with the series branches, compensated face
sum, epilogue) followed by pft_backward_3d (vertex adjoint) for a seeded
synthetic cotangent, both in the FP32-compensated form. The same step in the
FP64 form is timed as the GPU baseline, and the FP64 CPU oracle is timed on a
bounded sample of the same workload.

Prints one JSON line. Metric: face*Q evaluations per second of a fwd+bwd step.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Operation counts per (triangle, Q) pair (multiply or add = 1, FMA = 2; sin, cos, reciprocal = 1 each):
#   forward  = 104 flop (algorithmic): one face term of the edge sum with all three edges evaluated
#              (cross and dot products with Q, three edge sincs, two half-vertex phases, the
#              face-origin phase, the complex products and the accumulation); the kernel's edge sharing
#              and polynomial sinc do less work for the same result, which this count credits;
#   adjoint  = 165.8 flop: on this workload every pair takes the adjoint's small-phase branch (largest
#              centred vertex phase 2.07 < 3), where a face's barycentric moments are sums of complete
#              homogeneous symmetric polynomials of its vertex phases; the basis is the hardware count
#              (SQ_INSTS_VALU_FLOPS_FP32, _TRANS and _FP64 on the 5120-face sphere x 64^3 grid) of the adjoint
#              with those sums taken as their Taylor series to binary32 accuracy (stopped once m^n/n! < 1e-6).
#              The kernel evaluates the same moments, at the same error, from fitted polynomials of exp(ix)
#              of lower degree and executes fewer operations (its own count is reported beside the fraction
#              as counted_flop_per_face_q), which this basis credits as the forward's 104 credits its edge
#              sharing; the differentiated edge-sum branch, not run here, would count 200;
#   grad_Q   = 246 flop: the adjoint's recomputed terms (66), edge derivatives (15)
#              and edge products (25), two barycentric moments with their
#              normalisation and the face integral (59), Q.N and its phase (7),
#              the corner-weighted moment vector (42) and the accumulation of A
#              and B (32).
FLOP_FWD = 104.0
FLOP_BWD = 165.8
FLOP_DQ = 246.0
FLOP_2D = 21.0    # per edge-Q pair of the 2D edge sum (binary64)
PEAK_FP32_TFLOPS = 157.3   # MI355X FP32 vector (AMD published)
PEAK_FP64_TFLOPS = 78.6
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
KERNEL_SOURCES = os.path.join(ROOT, "paper_2104_08309_amd", "csrc")


def kernel_source_digest():
    """sha256 over the HIP and C++ sources: ties a traffic measurement to the code it was taken on."""
    import hashlib

    h = hashlib.sha256()
    for name in sorted(os.listdir(KERNEL_SOURCES)):
        if not name.endswith((".hip", ".h", ".cpp")):
            continue
        with open(os.path.join(KERNEL_SOURCES, name), "rb") as f:
            h.update(name.encode())
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary, or None if stale."""
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.loads(f.read())
    except (OSError, ValueError):
        return None
    if rec.get("source_digest") != kernel_source_digest():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("bytes_per_launch")


COUNTER_FILE = os.path.join(ROOT, "profiles", "valu_counters_icosphere_L4_grid64.txt")
COUNTER_SECTIONS = {"fwd3d_fp32c": "## fwd3d_fp32c_kernel<true", "bwd3d_fp32c": "## bwd3d_fp32c"}


def measured_flops(kernel):
    """FLOPs per (face, Q) pair that the hardware counters counted for `kernel` (FP32 + transcendental
    + FP64, FMA = 2) in the committed counter summary, or None if stale."""
    try:
        with open(COUNTER_FILE) as f:
            text = f.read()
    except OSError:
        return None
    if f"Kernel sources digest: {kernel_source_digest()}." not in text:
        return None
    head = COUNTER_SECTIONS.get(kernel)
    if head is None or head not in text:
        return None
    section = text.split(head, 1)[1].split("\n## ", 1)[0]
    for line in section.splitlines():
        if "counted FLOPs" in line:
            return float(line.rsplit("=", 1)[1])
    return None


def _oracle_chunk(args):
    """CPU-baseline worker: the oracle's forward and gradient on one Q chunk."""
    v, t, q, g = args
    import oracle as O

    t0 = time.perf_counter()
    F = O.ft3d(v, t, q)
    t1 = time.perf_counter()
    G = O.grad3d(v, t, q, g)
    t2 = time.perf_counter()
    return F, G, t1 - t0, t2 - t1


def _worker_init():
    """One BLAS thread per worker process (the pool supplies the parallelism) and the oracle imported
    before any timed work."""
    sys.path.insert(0, ROOT)
    from threadpoolctl import threadpool_limits

    global _BLAS_LIMIT
    _BLAS_LIMIT = threadpool_limits(limits=1)
    import oracle  # noqa: F401


def _ready(_):
    return os.getpid()


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(v, t, q_sample, g_sample, runs=3):
    """The oracle on a Q sample over a process pool of the host's cores (at most 16: the share of the
    host that one GPU's job gets), started and warmed before the clock runs; the median of `runs` runs."""
    import multiprocessing as mp

    cores = min(len(os.sched_getaffinity(0)), 16)
    n_chunks = 4 * cores
    chunks = [(v, t, qc, gc) for qc, gc in zip(np.array_split(q_sample, n_chunks), np.array_split(g_sample, n_chunks))]
    walls = []
    with mp.get_context("spawn").Pool(cores, initializer=_worker_init) as pool:
        pool.map(_ready, range(4 * cores), chunksize=1)
        for _ in range(runs):
            t0 = time.perf_counter()
            res = pool.map(_oracle_chunk, chunks, chunksize=1)
            walls.append(time.perf_counter() - t0)
    F = np.concatenate([r[0] for r in res])
    G = sum(r[1] for r in res)
    return F, G, float(np.median(walls)), walls, cores


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=4096, help="Q points of the oracle's timed sample")
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 GPU baseline")
    ap.add_argument("--no-orient", action="store_true", help="skip the orientation-average measurement")
    ap.add_argument("--no-poly", action="store_true", help="skip the polygon-face measurement")
    ap.add_argument("--no-loss", action="store_true", help="skip the fused intensity-loss measurement (config 4)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched (config 5) and 2D (config 1) measurements")
    ap.add_argument("--no-config3", action="store_true", help="skip the union-of-spheres forward (config 3)")
    ap.add_argument("--no-regions", action="store_true",
                    help="skip the grad_Q and multi-region (piecewise-constant density) measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the transform would shard by Q across "
              f"GPUs, but only the single-MI355X path is implemented and reported.", file=sys.stderr)
        sys.exit(2)

    import torch

    import meshgen as mg
    from paper_2104_08309_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2104_08309_amd import build as _b
        _b.build()
    import paper_2104_08309_amd as pft

    dev = torch.device("cuda:0")
    cfg = mg.config2()
    v, t, q = cfg["verts"], cfg["tris"], cfg["q"]
    nf, nq, nv = t.shape[0], q.shape[0], v.shape[0]
    rng = np.random.default_rng(2)
    g = (rng.normal(size=nq) + 1j * rng.normal(size=nq)) / nq

    V = torch.tensor(v, dtype=torch.float32, device=dev)
    V64 = torch.tensor(v, dtype=torch.float64, device=dev)
    T = torch.tensor(t, dtype=torch.int32, device=dev)
    Q = torch.tensor(q, dtype=torch.float32, device=dev)
    Q64 = torch.tensor(q, dtype=torch.float64, device=dev)
    G = torch.tensor(g.astype(np.complex64), device=dev)
    G64 = torch.tensor(g, device=dev)

    def step32():
        # the face order and the Q order are computed at the first call (warmup) and reused, as in a
        # fitting loop over a fixed mesh connectivity and Q set
        F = pft.forward_3d(V, T, Q, mode="fp32c")
        dV = pft.backward_3d(V, T, Q, G, mode="fp32c")
        return F, dV

    def step32_plain():
        # the same step with the list order of faces and a Q sort inside every call
        F = pft.forward_3d(V, T, Q, mode="fp32c", order=None, q_order=None)
        dV = pft.backward_3d(V, T, Q, G, mode="fp32c", q_order=None)
        return F, dV

    def step64():
        F = pft.forward_3d(V64, T, Q64, mode="fp64")
        dV = pft.backward_3d(V64, T, Q64, G64, mode="fp64")
        return F, dV

    def timed(fn, steps, warmup, per_step=None):
        """Mean wall time of `steps` calls bracketed by synchronisations; with a list `per_step`, also
        each call's time from HIP events on the current stream (no synchronisation in between)."""
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        pft.profile_reset()
        pft.profile_enable(True)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)] if per_step is not None else None
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if ev:
            ev[0].record()
        for i in range(steps):
            out = fn()
            if ev:
                ev[i + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        pft.profile_enable(False)
        if ev:
            per_step.extend(ev[i].elapsed_time(ev[i + 1]) for i in range(steps))
        return wall / steps, out

    print(f"[bench] fp32c fwd+bwd, {args.steps} steps", file=sys.stderr, flush=True)
    step_ms = []
    dt32, (F32, dV32) = timed(step32, args.steps, args.warmup, per_step=step_ms)
    n_f, ms_f = pft.profile_read("fwd3d_fp32c")
    n_b, ms_b = pft.profile_read("bwd3d_fp32c")
    fwd_ms, bwd_ms = ms_f / max(n_f, 1), ms_b / max(n_b, 1)
    value = nf * nq / dt32
    dt32p, _ = timed(step32_plain, max(3, args.steps // 4), 1)

    fp64 = None
    F64 = None
    if not args.no_fp64:
        steps64 = max(3, args.steps // 4)
        print(f"[bench] fp64 fwd+bwd, {steps64} steps", file=sys.stderr, flush=True)
        dt64, (F64, dV64) = timed(step64, steps64, 1)
        n_f6, ms_f6 = pft.profile_read("fwd3d_fp64")
        n_b6, ms_b6 = pft.profile_read("bwd3d_fp64")
        F64 = F64.cpu().numpy()
        dV64 = dV64.cpu().numpy()
        fp64 = {"value": nf * nq / dt64, "ms_per_step": dt64 * 1e3, "fwd_kernel_ms": ms_f6 / max(n_f6, 1),
                "bwd_kernel_ms": ms_b6 / max(n_b6, 1)}

    F32h = F32.cpu().numpy().astype(np.complex128)
    dV32h = dV32.cpu().numpy().astype(np.float64)
    acc = {}
    if F64 is not None:
        acc["fwd_rel_err_vs_fp64_gpu"] = float(np.linalg.norm(F32h - F64) / np.linalg.norm(F64))
        acc["bwd_rel_err_vs_fp64_gpu"] = float(np.linalg.norm(dV32h - dV64) / np.linalg.norm(dV64))

    if args.copy_calibration:
        src = torch.ones(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # orientation-averaged intensity on the same mesh: 256 magnitudes in (0, 0.5] x a 32 x 32 direction
    # rule, i.e. the same 262144 face-Q work per call as the forward above (FP32C and FP64 forms)
    orient = None
    if not args.no_orient:
        print("[bench] orientation average", file=sys.stderr, flush=True)
        qabs = np.linspace(0.5 / 256, 0.5, 256)
        dirs, wts = mg.sphere_quadrature(32, 32)
        qa_t = torch.tensor(qabs, device=dev)
        d_t = torch.tensor(dirs, device=dev)
        w_t = torch.tensor(wts, device=dev)

        def orient_call(mode):
            return pft.orientation_average(V64, T, qa_t, d_t, w_t, mode=mode)

        o_steps = max(3, args.steps // 4)
        t32, I32 = timed(lambda: orient_call("fp32c"), o_steps, 1)
        t64, I64 = timed(lambda: orient_call("fp64"), max(2, o_steps // 2), 1)
        I32, I64 = I32.cpu().numpy(), I64.cpu().numpy()
        npair = nf * qabs.size * dirs.shape[0]
        orient = {"workload": f"icosphere L4 mesh, {qabs.size} |Q| in (0, 0.5] x {dirs.shape[0]} directions "
                              f"(Gauss-Legendre 32 x uniform 32)",
                  "value_fp32c": npair / t32, "ms_per_call_fp32c": t32 * 1e3,
                  "value_fp64": npair / t64, "ms_per_call_fp64": t64 * 1e3, "unit": "face*Q/s",
                  "rel_err_fp32c_vs_fp64_gpu": float(np.linalg.norm(I32 - I64) / np.linalg.norm(I64))}
        if not args.no_cpu_baseline:
            import oracle as O
            pick = [37]
            Io = O.orientation_average(v, t, qabs[pick], dirs, wts)
            orient["rel_err_fp32c_vs_oracle_sample"] = float(np.max(np.abs(I32[pick] - Io) / np.abs(Io)))
            orient["oracle_sample"] = f"|Q| = {qabs[pick[0]]:.5f}, all {dirs.shape[0]} directions"

    # planar polygon faces: a lat-long sphere of radius 50 with 2496 quads and 128 pole triangles
    # (5120 triangles when fan-triangulated, as config 2's mesh), on config 2's Q grid, native
    # polygon kernel against the triangle kernel on the fan triangulation
    poly = None
    if not args.no_poly:
        print("[bench] polygon faces", file=sys.stderr, flush=True)
        pv, pf = mg.ellipsoid_quads([50.0, 50.0, 50.0], 42, 64)
        ptri = np.array([[x[0], x[l], x[l + 1]] for x in pf for l in range(1, len(x) - 1)], dtype=np.int32)
        PV = torch.tensor(pv, dtype=torch.float32, device=dev)
        PT = torch.tensor(ptri, device=dev)
        p_steps = max(3, args.steps // 4)
        tp, Fp = timed(lambda: pft.forward_3d_poly(PV, pf, Q, mode="fp32c"), p_steps, 1)
        n_p, ms_p = pft.profile_read("fwdpoly_fp32c")
        tt, Ft = timed(lambda: pft.forward_3d(PV, PT, Q, mode="fp32c"), p_steps, 1)
        n_t, ms_t = pft.profile_read("fwd3d_fp32c")
        n_edges = sum(len(x) for x in pf)
        Fp, Ft = Fp.cpu().numpy().astype(np.complex128), Ft.cpu().numpy().astype(np.complex128)
        poly = {"workload": f"lat-long sphere R=50: {len(pf)} planar faces ({n_edges} edges; {ptri.shape[0]} "
                            f"triangles when fan-triangulated) x config 2's {nq} Q, FP32C forward",
                "poly_kernel_ms": ms_p / max(n_p, 1), "tri_kernel_ms": ms_t / max(n_t, 1),
                "poly_ms_per_call": tp * 1e3, "tri_ms_per_call": tt * 1e3,
                "poly_edge_q_per_s": n_edges * nq / (ms_p / max(n_p, 1) * 1e-3),
                "rel_diff_poly_vs_triangles": float(np.linalg.norm(Fp - Ft) / np.linalg.norm(Ft))}

    # grad_Q F on config 2 (the dL/dQ kernel, FP32C and FP64) and a three-region layered sphere
    # (core R=30, shells to R=40 and R=50, level-4 icospheres: 25600 faces) on config 2's Q grid
    gradq = regions = None
    if not args.no_regions:
        print("[bench] grad_Q and regions", file=sys.stderr, flush=True)
        one = torch.ones(1, dtype=torch.float64, device=dev)
        r_steps = max(3, args.steps // 4)
        tq32, (_, _, GQ32) = timed(lambda: pft.backward_3d_regions(V, T, [0, nf], one, Q, G, mode="fp32c",
                                                                    need_verts=False, need_rho=False), r_steps, 1)
        n_q, ms_q = pft.profile_read("dq3d_fp32c")
        tq64, (_, _, GQ64) = timed(lambda: pft.backward_3d_regions(V64, T, [0, nf], one, Q64, G64, mode="fp64",
                                                                    need_verts=False, need_rho=False),
                                   max(2, r_steps // 2), 1)
        n_q6, ms_q6 = pft.profile_read("dq3d_fp64")
        GQ32, GQ64 = GQ32.cpu().numpy().astype(np.float64), GQ64.cpu().numpy()
        dq_ms, dq64_ms = ms_q / max(n_q, 1), ms_q6 / max(n_q6, 1)
        achieved = FLOP_DQ * nf * nq / (dq_ms * 1e-3) / 1e12
        gradq = {"workload": f"config 2 mesh x {nq} Q, dL/dQ = Re(conj(g) grad_Q F)",
                 "kernel_ms_fp32c": dq_ms, "kernel_ms_fp64": dq64_ms, "ms_per_call_fp32c": tq32 * 1e3,
                 "ms_per_call_fp64": tq64 * 1e3, "face_q_per_s_fp32c": nf * nq / (dq_ms * 1e-3),
                 "speedup_fp32c_vs_fp64_kernel": dq64_ms / dq_ms,
                 "alu": {"achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                         "frac": achieved / PEAK_FP32_TFLOPS, "flop_per_face_q": FLOP_DQ},
                 "rel_err_fp32c_vs_fp64_gpu": float(np.linalg.norm(GQ32 - GQ64) / np.linalg.norm(GQ64))}
        lv, lt, loff = mg.layered_sphere(4, [30.0, 40.0, 50.0])
        LV = torch.tensor(lv, dtype=torch.float32, device=dev)
        LT = torch.tensor(lt, dtype=torch.int32, device=dev)
        rho_h = np.array([1.0, 0.6, 0.85])
        RHO = torch.tensor(rho_h, device=dev)
        tf, (FR, FRj) = timed(lambda: pft.forward_3d_regions(LV, LT, loff, RHO, Q, mode="fp32c", per_region=True),
                              r_steps, 1)
        n_rf, ms_rf = pft.profile_read("fwd3d_fp32c")
        tb, _ = timed(lambda: pft.backward_3d_regions(LV, LT, loff, RHO, Q, G, mode="fp32c"), r_steps, 1)
        n_rb, ms_rb = pft.profile_read("bwd3d_fp32c")
        n_rq, ms_rq = pft.profile_read("dq3d_fp32c")
        nfl = lt.shape[0]
        regions = {"workload": f"layered sphere: core R=30 and shells to R=40, R=50 (level-4 icospheres, {nfl} "
                               f"faces in 3 regions) x config 2's {nq} Q, FP32C",
                   "forward_kernel_ms": ms_rf / max(n_rf, 1), "forward_ms_per_call": tf * 1e3,
                   "forward_face_q_per_s": nfl * nq / (ms_rf / max(n_rf, 1) * 1e-3),
                   "backward_ms_per_call": tb * 1e3, "adjoint_kernel_ms": ms_rb / max(n_rb, 1),
                   "grad_q_kernel_ms": ms_rq / max(n_rq, 1),
                   "backward_outputs": "dL/dverts, dL/drho, dL/dQ"}
        if not args.no_cpu_baseline:
            import oracle as O
            srng = np.random.default_rng(13)
            pick = np.concatenate([[int(np.argmin(np.linalg.norm(q, axis=1)))], srng.choice(nq, 255, replace=False)])
            gq_o = np.real(np.conj(G.cpu().numpy().astype(np.complex128)[pick])[:, None]
                           * O.ft3d_dq(v.astype(np.float32).astype(np.float64), t,
                                       q[pick].astype(np.float32).astype(np.float64)))
            gradq["rel_err_fp32c_vs_oracle_sample"] = float(np.linalg.norm(GQ32[pick] - gq_o) / np.linalg.norm(gq_o))
            gradq["oracle_sample"] = "256 grid Q incl. Q = 0, all faces"
            pr = pick[:64]
            Fo, _ = O.ft3d_regions(lv.astype(np.float32).astype(np.float64), lt, loff, rho_h,
                                   q[pr].astype(np.float32).astype(np.float64))
            FRh = FR.cpu().numpy().astype(np.complex128)
            regions["forward_rel_err_vs_oracle_sample"] = float(np.linalg.norm(FRh[pr] - Fo) / np.linalg.norm(Fo))
            regions["oracle_sample"] = "64 grid Q incl. Q = 0, all faces"

    # the adjoint's workload (config 4: icosphere L6 with 2 % radial noise, 256^2 Q slice) as a fitting step:
    # L = sum w (|F|^2 - I)^2 against the sphere's intensity and dL/dv, fused in one library call, against the
    # same step through forward_3d, the loss in torch and backward_3d
    lossf = None
    if not args.no_loss:
        print("[bench] fused intensity loss (config 4)", file=sys.stderr, flush=True)
        c4 = mg.config4()
        V4 = torch.tensor(c4["verts"], dtype=torch.float32, device=dev)
        T4 = torch.tensor(c4["tris"], dtype=torch.int32, device=dev)
        Q4 = torch.tensor(c4["q"], dtype=torch.float32, device=dev)
        x = np.linalg.norm(c4["q"], axis=1) * c4["radius"]
        vol = 4.0 / 3.0 * np.pi * c4["radius"] ** 3
        with np.errstate(invalid="ignore", divide="ignore"):
            form = np.where(x < 1e-3, 1.0 - x * x / 10.0, 3.0 * (np.sin(x) - x * np.cos(x)) / x ** 3)
        I4 = torch.tensor((vol * form) ** 2, device=dev)
        W4 = torch.full((len(x),), 1.0 / (len(x) * vol ** 4), dtype=torch.float64, device=dev)

        def fused():
            return pft.intensity_loss_3d(V4, T4, Q4, I4, W4, mode="fp32c")

        def unfused():
            F = pft.forward_3d(V4, T4, Q4, mode="fp32c").to(torch.complex128)
            r = F.real ** 2 + F.imag ** 2 - I4
            L = torch.sum(W4 * r * r)
            return L, pft.backward_3d(V4, T4, Q4, (4.0 * W4 * r * F).to(torch.complex64), mode="fp32c")

        l_steps = max(3, args.steps // 4)
        tfu, (Lf, Gf) = timed(fused, l_steps, 1)
        n_lf, ms_lf = pft.profile_read("fwd3d_fp32c")
        n_lb, ms_lb = pft.profile_read("bwd3d_fp32c")
        tun, (Lu, Gu) = timed(unfused, l_steps, 1)
        Gf, Gu = Gf.cpu().numpy().astype(np.float64), Gu.cpu().numpy().astype(np.float64)
        nf4, nq4 = c4["tris"].shape[0], len(x)
        lossf = {"workload": f"config 4: icosphere L6 with 2% radial noise ({nf4} faces) x 256^2 Q slice, "
                             f"L = sum w (|F|^2 - I_sphere)^2 and dL/dv, FP32C",
                 "fused_ms_per_step": tfu * 1e3, "unfused_ms_per_step": tun * 1e3,
                 "fused_face_q_per_s": nf4 * nq4 / tfu,
                 "forward_kernel_ms": ms_lf / max(n_lf, 1), "adjoint_kernel_ms": ms_lb / max(n_lb, 1),
                 "loss_rel_diff_fused_vs_unfused": abs(Lf.item() - Lu.item()) / abs(Lu.item()),
                 "grad_rel_diff_fused_vs_unfused": float(np.linalg.norm(Gf - Gu) / np.linalg.norm(Gu))}
        # accuracy against the FP64 form: the adjoint alone (both forms on one cotangent, the loss's, formed
        # from the FP64 forward) and end to end (each form's own fused loss gradient). The end-to-end error
        # is the FP32C forward's error passed through the loss ("cotangent error": the FP64 adjoint of the
        # cotangent formed from the FP32C F) plus the adjoint's own.
        V4d, Q4d = V4.double(), Q4.double()
        L64, G64, F64 = pft.intensity_loss_3d(V4d, T4, Q4d, I4, W4, mode="fp64", return_F=True)
        L32, G32, F32 = pft.intensity_loss_3d(V4, T4, Q4, I4, W4, mode="fp32c", return_F=True)
        F32 = F32.to(torch.complex128)

        def cot(F):
            return 4.0 * W4 * (F.real ** 2 + F.imag ** 2 - I4) * F

        g64 = cot(F64).to(torch.complex64)
        A32 = pft.backward_3d(V4, T4, Q4, g64, mode="fp32c").double()
        A64 = pft.backward_3d(V4d, T4, Q4d, g64.to(torch.complex128), mode="fp64")
        Gc = pft.backward_3d(V4d, T4, Q4d, cot(F32), mode="fp64")

        def nrel(a, b):
            return float(torch.linalg.norm(a.double() - b.double()) / torch.linalg.norm(b.double()))

        e_F, e_c, e_g = nrel(F32, F64), nrel(Gc, G64), nrel(G32, G64)
        lossf.update({"forward_rel_err_fp32c_vs_fp64": e_F,
                      "adjoint_rel_err_same_cotangent_fp32c_vs_fp64": nrel(A32, A64),
                      "grad_rel_err_fp32c_vs_fp64": e_g,
                      "cotangent_error_through_adjoint": e_c,
                      "loss_amplification_of_forward_error": e_c / e_F,
                      "loss_rel_err_fp32c_vs_fp64": abs(L32.item() - L64.item()) / abs(L64.item())})
        del V4d, Q4d, F64, F32, G64, G32, A32, A64, Gc

    # config 5 (512 uneven meshes, one persistent launch each way) and config 1 (the 2D path, binary64)
    batch = fwd2d = None
    if not args.no_batch:
        print("[bench] batch (config 5) and 2D (config 1)", file=sys.stderr, flush=True)
        meshes = mg.config5()
        vo, to, qo = [0], [0], [0]
        for m in meshes:
            vo.append(vo[-1] + len(m["verts"]))
            to.append(to[-1] + len(m["tris"]))
            qo.append(qo[-1] + len(m["q"]))
        BV = torch.tensor(np.concatenate([m["verts"] for m in meshes]), dtype=torch.float32, device=dev)
        BT = torch.tensor(np.concatenate([m["tris"] for m in meshes]), dtype=torch.int32, device=dev)
        BQ = torch.tensor(np.concatenate([m["q"] for m in meshes]), dtype=torch.float32, device=dev)
        brng = np.random.default_rng(5)
        bg = (brng.normal(size=qo[-1]) + 1j * brng.normal(size=qo[-1])) / qo[-1]
        BG = torch.tensor(bg.astype(np.complex64), device=dev)
        pairs = sum(len(m["tris"]) * len(m["q"]) for m in meshes)

        def bstep():
            return (pft.batch_forward(BV, BT, BQ, vo, to, qo, mode="fp32c"),
                    pft.batch_backward(BV, BT, BQ, vo, to, qo, BG, mode="fp32c"))

        b_steps = max(2, args.steps // 8)
        # the first (warmup) call tunes the tile sizes for this input's size bucket; then the same step
        # with the compiled default tile sizes
        tb5, (BF, BD) = timed(bstep, b_steps, 1)
        n_bf, ms_bf = pft.profile_read("batch_fwd")
        n_bb, ms_bb = pft.profile_read("batch_bwd")
        ms_bf, ms_bb = ms_bf / max(n_bf, 1), ms_bb / max(n_bb, 1)
        os.environ["PFT_AUTOTUNE"] = "0"
        tb5d, _ = timed(bstep, b_steps, 1)
        n_df, ms_df = pft.profile_read("batch_fwd")
        n_db, ms_db = pft.profile_read("batch_bwd")
        del os.environ["PFT_AUTOTUNE"]
        batch = {"workload": f"config 5: {len(meshes)} meshes, {to[-1]} faces, {qo[-1]} Q, {pairs:.3e} face*Q "
                             f"(each mesh its own Q list), FP32C forward + adjoint, one persistent launch each",
                 "ms_per_step": tb5 * 1e3, "face_q_per_s": pairs / tb5,
                 "forward_kernel_ms": ms_bf, "adjoint_kernel_ms": ms_bb,
                 "forward_alu_frac": FLOP_FWD * pairs / (ms_bf * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                 "adjoint_alu_frac": FLOP_BWD * pairs / (ms_bb * 1e-3) / 1e12 / PEAK_FP32_TFLOPS,
                 "tuned_tiles": pft.tuning_info().strip().split("\n"),
                 "default_tiles_ms_per_step": tb5d * 1e3,
                 "default_tiles_forward_kernel_ms": ms_df / max(n_df, 1),
                 "default_tiles_adjoint_kernel_ms": ms_db / max(n_db, 1)}
        c1 = mg.config1()
        P2 = torch.tensor(c1["verts"], device=dev)
        Q2d = torch.tensor(c1["q"], device=dev)
        t2, F2 = timed(lambda: pft.forward_2d(P2, Q2d), max(10, args.steps), 2)
        n_2, ms_2 = pft.profile_read("fwd2d_fp64")
        ne, nq2 = c1["verts"].shape[0], c1["q"].shape[0]
        k2 = ms_2 / max(n_2, 1)
        fwd2d = {"workload": f"config 1: star polygon, {ne} edges x {nq2} Q (128^2 grid over [-20,20)^2), binary64",
                 "ms_per_call": t2 * 1e3, "kernel_ms": k2, "edge_q_per_s": ne * nq2 / t2,
                 "fp64_alu_frac": FLOP_2D * ne * nq2 / (k2 * 1e-3) / 1e12 / PEAK_FP64_TFLOPS}
        if not args.no_cpu_baseline:
            import oracle as O
            F2o = O.ft2d(c1["verts"], c1["q"])
            fwd2d["rel_err_vs_oracle"] = float(np.linalg.norm(F2.cpu().numpy() - F2o) / np.linalg.norm(F2o))
            # the four meshes with the least work, every Q: forward and adjoint against the oracle
            order = np.argsort([len(m["tris"]) * len(m["q"]) for m in meshes])[:4]
            BFh = BF.cpu().numpy().astype(np.complex128)
            BDh = BD.cpu().numpy().astype(np.float64)
            ef, eb = [], []
            for i in order:
                m = meshes[i]
                vm = m["verts"].astype(np.float32).astype(np.float64)
                qm = m["q"].astype(np.float32).astype(np.float64)
                Fo = O.ft3d(vm, m["tris"], qm)
                ef.append(float(np.linalg.norm(BFh[qo[i]:qo[i + 1]] - Fo) / np.linalg.norm(Fo)))
                Go = O.grad3d(vm, m["tris"], qm, bg.astype(np.complex64)[qo[i]:qo[i + 1]])
                eb.append(float(np.linalg.norm(BDh[vo[i]:vo[i + 1]] - Go) / np.linalg.norm(Go)))
            batch["forward_rel_err_vs_oracle_4_meshes"] = max(ef)
            batch["adjoint_rel_err_vs_oracle_4_meshes"] = max(eb)

    # config 3: the union of 20 spheres (about 1e5 faces) x a 128^3 Q grid, FP32C forward with |F|^2
    union = None
    if not args.no_config3:
        print("[bench] union of spheres (config 3)", file=sys.stderr, flush=True)
        c3 = mg.config3()
        V3 = torch.tensor(c3["verts"], dtype=torch.float32, device=dev)
        T3 = torch.tensor(c3["tris"], dtype=torch.int32, device=dev)
        Q3 = torch.tensor(c3["q"], dtype=torch.float32, device=dev)
        t3, (F3, I3) = timed(lambda: pft.forward_3d(V3, T3, Q3, mode="fp32c", intensity=True), 2, 1)
        n_3, ms_3 = pft.profile_read("fwd3d_fp32c")
        ms_3 = ms_3 / max(n_3, 1)
        nf3, nq3 = c3["tris"].shape[0], c3["q"].shape[0]
        union = {"workload": f"config 3: union of 20 spheres ({nf3} faces) x 128^3 Q over [-0.3,0.3)^3, FP32C "
                             f"forward with |F|^2 (edge-sharing order)",
                 "ms_per_call": t3 * 1e3, "kernel_ms": ms_3, "face_q_per_s": nf3 * nq3 / t3,
                 "alu_frac": FLOP_FWD * nf3 * nq3 / (ms_3 * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}
        if not args.no_cpu_baseline:
            import oracle as O
            srng = np.random.default_rng(14)
            pick = np.concatenate([[int(np.argmin(np.linalg.norm(c3["q"], axis=1)))], srng.choice(nq3, 63, replace=False)])
            Fo3 = O.ft3d(c3["verts"].astype(np.float32).astype(np.float64), c3["tris"],
                         c3["q"][pick].astype(np.float32).astype(np.float64))
            F3h = F3.cpu().numpy().astype(np.complex128)[pick]
            union["rel_err_vs_oracle_sample"] = float(np.linalg.norm(F3h - Fo3) / np.linalg.norm(Fo3))
            union["max_err_over_max_F_sample"] = float(np.max(np.abs(F3h - Fo3)) / np.max(np.abs(Fo3)))
            union["oracle_sample"] = "64 grid Q incl. Q = 0, all faces"
        del V3, T3, Q3, F3, I3

    # roofline of the dominant kernel (the longer of the forward and adjoint kernels)
    def roof(kernel, ms, flop):
        achieved = flop * nf * nq / (ms * 1e-3) / 1e12
        counted = measured_flops(kernel)
        return {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(kernel), "kernel": kernel,
                "kernel_ms": ms, "flop_per_face_q": flop, "launch_face_q": nf * nq,
                # what the kernel executes per pair (hardware count), and the fraction at that count
                "counted_flop_per_face_q": counted,
                "frac_at_counted": None if counted is None else
                counted * nf * nq / (ms * 1e-3) / 1e12 / PEAK_FP32_TFLOPS}

    r_fwd = roof("fwd3d_fp32c", fwd_ms, FLOP_FWD)
    r_bwd = roof("bwd3d_fp32c", bwd_ms, FLOP_BWD)
    roofline, other = (r_bwd, r_fwd) if bwd_ms >= fwd_ms else (r_fwd, r_bwd)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu baseline (oracle)", file=sys.stderr, flush=True)
        srng = np.random.default_rng(12)
        special = np.nonzero((np.sum(q != 0, axis=1) <= 1) | ((q[:, 0] == q[:, 1]) & (q[:, 1] == q[:, 2])))[0]
        idx = np.unique(np.concatenate([special[:: max(1, special.size // 64)],
                                        srng.choice(nq, args.cpu_sample, replace=False)]))[: args.cpu_sample]
        qs = q[idx]
        gs = g[idx]
        Fo, Go, wall, walls, cores = cpu_baseline(v, t, qs, gs)
        cpu = {"value": nf * qs.shape[0] / wall, "unit": "face*Q/s (fwd+bwd)", "cores": cores, "kind": "oracle",
               "sample": f"{qs.shape[0]} of the {nq} grid Q (seeded, incl. Q=0, axes, diagonal), all {nf} faces, "
                         f"forward + vertex gradient; median of {len(walls)} runs "
                         f"({', '.join(f'{w:.1f}' for w in walls)} s wall) on a pool started beforehand",
               "runs_s": walls}
        acc["fwd_rel_err_vs_oracle_sample"] = float(np.linalg.norm(F32h[idx] - Fo) / np.linalg.norm(Fo))
        acc["fwd_max_err_over_max_F_sample"] = float(np.max(np.abs(F32h[idx] - Fo)) / np.max(np.abs(Fo)))
        # the adjoint over the sample only: run the FP32C kernel on the same Q subset
        Gsub = pft.backward_3d(V, T, torch.tensor(qs, dtype=torch.float32, device=dev),
                               torch.tensor(gs.astype(np.complex64), device=dev), mode="fp32c").cpu().numpy()
        Go32 = Go  # oracle at float64 inputs; the kernel sees float32 Q and vertices
        acc["bwd_rel_err_vs_oracle_sample"] = float(np.linalg.norm(Gsub - Go32) / np.linalg.norm(Go32))
        acc["bwd_max_err_over_max_grad_sample"] = float(np.max(np.abs(Gsub - Go32)) / np.max(np.abs(Go32)))
        # one host core on a smaller sample of the same Q (the oracle as it stands, one process, one BLAS thread)
        from threadpoolctl import threadpool_limits
        sub = idx[: max(64, len(idx) // 8)]
        with threadpool_limits(limits=1):
            t1 = time.perf_counter()
            _oracle_chunk((v, t, q[sub], g[sub]))
            cpu["single_core_value"] = nf * len(sub) / (time.perf_counter() - t1)
        cpu["single_core_sample"] = f"{len(sub)} of the same Q, one process, one BLAS thread"
        cpu["single_core_times_cores"] = cpu["single_core_value"] * cores
        cpu["parallel_efficiency"] = cpu["value"] / cpu["single_core_times_cores"]
        cpu["cpu_model"] = _cpu_model()

    line = {
        "metric": "face*Q evals/sec fwd+bwd, FP32-compensated vs FP64 GPU at <=1e-5 rel err",
        "value": value,
        "unit": "face*Q/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt32 * 1e3,
        "ms_per_step_median": float(np.median(step_ms)),
        "ms_per_step_list_order_sorted_in_call": dt32p * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "dtype_note": "FP32-compensated: edge arithmetic in binary32, face phases, series branches and the "
                      "sums across tiles and splits in binary64",
        "data": "synthetic",
        "config": {"workload": "icosphere L4 (5120 tri, R=50), Q 64^3 grid over [-0.5,0.5)^3, fwd+bwd FP32C",
                   "faces": nf, "vertices": nv, "n_q": nq},
        "fwd_kernel_ms": fwd_ms,
        "bwd_kernel_ms": bwd_ms,
        "alu_frac_fwd": r_fwd["frac"],
        "alu_frac_bwd": r_bwd["frac"],
        "fp64_gpu": fp64,
        "speedup_vs_fp64_gpu": (fp64["ms_per_step"] / (dt32 * 1e3)) if fp64 else None,
        "accuracy": acc,
        "roofline": roofline,
        "roofline_other_kernel": other,
        "cpu_baseline": cpu,
        "orientation_average": orient,
        "polygon_faces": poly,
        "grad_q": gradq,
        "regions": regions,
        "intensity_loss": lossf,
        "kernel_source_digest": kernel_source_digest(),
        "host_cpu": _cpu_model(),
        "batch": batch,
        "forward_2d": fwd2d,
        "union_of_spheres": union,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
