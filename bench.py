"""Benchmark of the bilayer minimum-mode kernel on one MI355X.

Headline (the 128x128 three-shell workload, FP32 HVP):
  * tangent HVP throughput, G site-vectors/s, on a batch of B = 1024
    independent 128x128 lattices x 4 vectors in the FP32 frame layout (the
    footprint, 1.3 GB, is several times the 256 MB Infinity Cache, so the
    kernel streams from HBM); one step = one batched HVP launch;
  * the roofline of that kernel (algorithmic bytes 12 + 16 n_vec per site);
  * wall time of the k = 4 eigen-solve (residual 1e-5) on one 128x128 state;
  * a k = 8 solve on a 512x512 two-skyrmion state and k = 2 solves from
    16x16 to 1024x1024 (time and workspace against size);
  * the 35-shell Pd/Fe/Ir(111) exchange (360 bonds per site) HVP on 64
    128x128 lattices, against the VALU and LDS ceilings;
  * a population of 24 k = 2 eigen-solves in lock step against one at a
    time, and the explorer objectives of 24 candidates;
  * saddle searches/s (k = 2, FP32 HVP, tau_F = 1e-5, capped outer
    iterations): 64 searches on 128x128 in lock step over the whole chip and
    in one persistent launch, 256 on
    uneven 32..96 lattices in one launch, and searches one at a time
    (L-BFGS, and the nonlinear-CG outer rule on the same starts);
  * the FP64 CPU oracle timed on a bounded sample of the same HVP workload.

Prints one JSON line.  `--gpus N` with N > 1 is refused: the library and
this benchmark run on one GPU.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "tangent HVP Gsite/s (GB/s vs HBM peak) + saddle searches/s, 128² lattice"
HBM_PEAK_GBS = 8000.0


def hvp_inputs(M, S, torch, plan, L, B, nvec, n_distinct=32, seed=2025):
    """B states tiled from n_distinct seeded skyrmion/antiskyrmion starts;
    c from moto_energy_grad; random frame-coordinate vectors."""
    kinds = ["skyrmion", "antiskyrmion"]
    base = np.stack([S.three_shell_start(L, seed=seed + i, kind=kinds[i % 2]) for i in range(n_distinct)])
    base_t = torch.as_tensor(base, dtype=torch.float32, device="cuda")
    reps = (B + n_distinct - 1) // n_distinct
    m = base_t.repeat(reps, 1, 1)[:B].contiguous()
    _, _, c, _, _ = M.moto_energy_grad(plan, m, want_grad=False, want_F=False)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    V = torch.randn(B, nvec, 2, L * L, dtype=torch.float32, device="cuda", generator=gen)
    W = torch.empty_like(V)
    return m, c.contiguous(), V, W, base


def counter_traffic(variant, B, L, nvec):
    """HBM bytes per launch of `variant` from the committed rocprofv3 counter
    summary, or None when the workload differs or the kernel source changed
    since the counters were taken."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "hvp_frame_1024x128x128_counters.md")
    if (B, L, nvec) != (1024, 128, 4) or not os.path.exists(path):
        return None
    src = os.path.join(ROOT, "paper_2509_26269_amd", "csrc", "hvp.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    rec, tb = None, {}
    for line in open(path):
        t = line.strip()
        if t.startswith("source_sha256 hvp.hip = "):
            rec = t.split("= ", 1)[1]
        elif t.startswith("traffic_bytes "):
            k, v = t[len("traffic_bytes "):].rsplit(" = ", 1)
            tb[k] = int(v)
    return tb.get(variant) if rec == h else None


def copy_peak_gbs(torch, mib=1024, reps=5):
    """Device-to-device copy of `mib` MiB (read + write bytes / time)."""
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    del src, dst
    return 2 * n * 4 / (ms * 1e-3) / 1e9


def time_hvp(M, torch, plan, m, c, V, W, B, steps, warmup):
    for _ in range(warmup):
        M.moto_tangent_hvp(plan, m, c, V, M.MOTO_FRAME, W=W, batch=B)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record()
    for i in range(steps):
        ev[i][0].record()
        M.moto_tangent_hvp(plan, m, c, V, M.MOTO_FRAME, W=W, batch=B)
        ev[i][1].record()
    t1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    per = [a.elapsed_time(b) for a, b in ev]
    return t0.elapsed_time(t1), per, wall


def cpu_baseline(O, S, p, base, nvec, budget_s=12.0):
    """FP64 oracle HVP (frame coordinates in and out) on a bounded sample of
    the workload: distinct states x nvec vectors, until the time budget."""
    h = O.Ham(**p.asdict())
    rng = np.random.default_rng(7)
    n_done = 0
    t0 = time.perf_counter()
    i = 0
    while time.perf_counter() - t0 < budget_s:
        m = base[i % len(base)].astype(np.float64)
        m = m / np.linalg.norm(m, axis=0)
        _, _, c, _ = O.energy_grad(h, m)
        a = rng.standard_normal((nvec, 2, h.N))
        t1 = time.perf_counter()
        v = O.from_frame(m, a)
        w = O.tangent_hvp(h, m, c, v)
        _ = O.to_frame(m, w)
        n_done += nvec
        i += 1
        del t1
    el = time.perf_counter() - t0
    return n_done, el


def _cpu_worker(args):
    """One host process of the all-cores baseline: the FP64 oracle HVP on
    its share of the distinct seeded states (the recipe of hvp_inputs)."""
    wid, nproc, L, nvec, n_distinct, seed, budget_s = args
    sys.path.insert(0, ROOT)
    import oracle as O
    from paper_2509_26269_amd import synth as S

    h = O.Ham(**S.ham_3shell(L).asdict())
    kinds = ["skyrmion", "antiskyrmion"]
    rng = np.random.default_rng(7 + wid)
    n_done = 0
    t0 = time.perf_counter()
    i = wid
    while time.perf_counter() - t0 < budget_s:
        m = S.three_shell_start(L, seed=seed + i % n_distinct, kind=kinds[(i % n_distinct) % 2])
        _, _, c, _ = O.energy_grad(h, m)
        a = rng.standard_normal((nvec, 2, h.N))
        w = O.tangent_hvp(h, m, c, O.from_frame(m, a))
        _ = O.to_frame(m, w)
        n_done += nvec
        i += nproc
    return n_done, time.perf_counter() - t0


def cpu_baseline_all_cores(L, nvec, budget_s=12.0, n_distinct=32, seed=2025):
    """The same oracle sample spread over the host cores (one process each,
    spawned so that none inherits the GPU context); cores capped at 16."""
    import multiprocessing as mp

    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count() or 1
    ncores = max(1, min(ncores, 16))
    ctx = mp.get_context("spawn")
    with ctx.Pool(ncores) as pool:
        t0 = time.perf_counter()
        res = pool.map(_cpu_worker, [(w, ncores, L, nvec, n_distinct, seed, budget_s) for w in range(ncores)])
        wall = time.perf_counter() - t0
    n_done = sum(r[0] for r in res)
    el = max(r[1] for r in res)
    return n_done, el, ncores, wall


def _cpu_search_worker(args):
    """One host process of the oracle search baseline: the FP64 oracle climb
    (k = 2, tau_F = 1e-5) from one seeded 128x128 start of the lock-step
    search leg, for a bounded number of outer steps."""
    wid, L, n, max_outer = args
    sys.path.insert(0, ROOT)
    import oracle as O
    from paper_2509_26269_amd import synth as S

    h = O.Ham(**S.ham_3shell(L).asdict())
    m0 = S.batch_member(S.fixed_size_spec(n, L, seed=128), wid)
    t0 = time.perf_counter()
    r = O.saddle_search(h, m0, tau_F=1e-5, k=2, eig_tol=1e-5, max_outer=max_outer)
    return r.iters, time.perf_counter() - t0


def cpu_search_all_cores(L, max_outer, n_starts=64):
    """Oracle climbs from the first `cores` starts, one single-threaded
    process per core (spawned, cores capped at 16): outer iterations per
    second."""
    import multiprocessing as mp

    try:
        ncores = len(os.sched_getaffinity(0))
    except AttributeError:
        ncores = os.cpu_count() or 1
    ncores = max(1, min(ncores, 16, n_starts))
    # one BLAS / OpenMP thread per worker process: the oracle's dense steps
    # would otherwise start a thread per core in every process
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(ncores) as pool:
            res = pool.map(_cpu_search_worker, [(w, L, n_starts, max_outer) for w in range(ncores)])
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    its = sum(r[0] for r in res)
    el = max(r[1] for r in res)
    return its, el, ncores


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--batch", type=int, default=1024)
    ap.add_argument("--nvec", type=int, default=4)
    ap.add_argument("--L", type=int, default=128)
    ap.add_argument("--searches", type=int, default=2, help="one-at-a-time GPU searches timed")
    ap.add_argument("--searches-masked", type=int, default=8,
                    help="of the masked 128x128 starts, how many also run one at a time")
    ap.add_argument("--batched", type=int, default=64, help="searches on 128x128 in the batched (one-launch) leg")
    ap.add_argument("--ragged", type=int, default=256, help="searches on uneven 32..96 lattices, one launch")
    ap.add_argument("--max-outer", type=int, default=300, help="outer-iteration cap of the unmasked search legs")
    ap.add_argument("--max-outer-masked", type=int, default=600,
                    help="outer-iteration cap of the masked search legs")
    ap.add_argument("--ragged-single", type=int, default=8,
                    help="masked ragged searches also run one at a time (same starts, same tau_F)")
    ap.add_argument("--large", type=int, default=1, help="512x512 k=8 solve and the k=2 size sweep (0: skip)")
    ap.add_argument("--shells35", type=int, default=64,
                    help="lattices in the 35-shell (Pd/Fe/Ir(111)) HVP leg (0: skip)")
    ap.add_argument("--population", type=int, default=24,
                    help="population size of the lock-step eigen-solve and explorer legs (0: skip)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-search", action="store_true")
    ap.add_argument("--hvp-only", action="store_true", help="only the HVP leg (for profilers)")
    ap.add_argument("--eigen-only", action="store_true",
                    help="only the eigen-solve leg and the search legs asked for (for profilers)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="first run one plain device copy of this many MiB (byte-counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: runs on one GPU only; multi-GPU runs are not supported "
              "(independent lattices would shard across GPUs with no communication).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2509_26269_amd import moto as M
    from paper_2509_26269_amd import synth as S

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    L, B, nvec = args.L, args.batch, args.nvec
    if args.calib_copy_mib > 0:
        n = args.calib_copy_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {args.calib_copy_mib} MiB done", file=sys.stderr, flush=True)
        del src, dst
    p = S.ham_3shell(L)
    plan = M.Plan.from_params(p)
    N = L * L
    if args.eigen_only:
        B = 32
    print(f"[bench] inputs: {B} x {L}x{L}, n_vec={nvec}", file=sys.stderr, flush=True)
    m, c, V, W, base = hvp_inputs(M, S, torch, plan, L, B, nvec)
    torch.cuda.synchronize()
    out = {"metric": METRIC, "value": None, "unit": "Gsite/s", "n_gpus": 1, "note": "eigen-only profiling run"}
    if not args.eigen_only:
        print("[bench] autotuning the frame-layout HVP", file=sys.stderr, flush=True)
        chosen, vtimes = M.moto_tangent_hvp_autotune(plan, m, c, V, W, batch=B, reps=10)
        vname = M.lib().moto_tangent_hvp_variant_name(chosen).decode()
        print(f"[bench] variants (ms): {vtimes} -> {vname}", file=sys.stderr, flush=True)
        print("[bench] timing batched tangent HVP", file=sys.stderr, flush=True)
        total_ms, per, wall = time_hvp(M, torch, plan, m, c, V, W, B, args.steps, args.warmup)
        ms_per_step = total_ms / args.steps
        avg_launch_ms = float(np.mean(per))
        site_vecs = B * N * nvec
        gsites = site_vecs / (ms_per_step * 1e-3) / 1e9
        alg_bytes = (12 + 16 * nvec) * N * B
        achieved = alg_bytes / (avg_launch_ms * 1e-3) / 1e9
        traffic = counter_traffic(vname, B, L, nvec)
        copy_gbs = copy_peak_gbs(torch)
        out = {
            "metric": METRIC,
            "value": round(gsites, 3),
            "unit": "Gsite/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": round(ms_per_step, 5),
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f32",
            "data": "synthetic",
            "config": {
                "workload": f"tangent HVP, frame layout, batch of {B} periodic {L}x{L} triangular lattices "
                            f"x {nvec} vectors, 3 exchange shells + NN DMI + K + B (J2,J3 seeded), "
                            "seeded skyrmion/antiskyrmion states",
                "lattice": f"{L}x{L}", "batch": B, "n_vec": nvec, "hvp": "f32",
            },
            "roofline": {
                "bound": "hbm",
                "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS,
                "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": traffic,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "traffic_over_alg": round(traffic / alg_bytes, 4) if traffic else None,
                "measured_copy_GBps": round(copy_gbs, 1),
                "frac_of_copy": round(achieved / copy_gbs, 4),
                "kernel": f"frame-layout tangent HVP, variant {vname}",
                "autotune_ms": {k2: round(v2, 4) for k2, v2 in vtimes.items()},
                "alg_bytes_per_launch": alg_bytes,
                "avg_launch_ms": round(avg_launch_ms, 5),
                "launch_ms_p10_p50_p90": [round(float(np.percentile(per, q)), 5) for q in (10, 50, 90)],
            },
            "device": {"name": torch.cuda.get_device_name(0), "hip": torch.version.hip,
                       "compute_units": torch.cuda.get_device_properties(0).multi_processor_count},
        }
    del W, V, m, c
    torch.cuda.empty_cache()

    extra = {}
    if not args.hvp_only:
        # eigen-solve wall time on one 128x128 state (k = 4, residual 1e-5)
        print("[bench] 128x128 k=4 FP32 eigen-solve", file=sys.stderr, flush=True)
        m1 = torch.as_tensor(base[0].astype(np.float64), device="cuda")
        m1 = m1 / m1.norm(dim=0, keepdim=True)
        # the library's default options (guard 8 for k = 4, cap 200)
        ws = M.EigWorkspace(plan, M.MOTO_F32, 4)
        o = M.eig_opts(M.MOTO_F32, tol=1e-5)
        r = M.moto_min_modes(plan, m1, 4, M.MOTO_F32, opts=o, ws=ws)
        torch.cuda.synchronize()
        times = []
        for _ in range(5):
            t0 = time.perf_counter()
            r = M.moto_min_modes(plan, m1, 4, M.MOTO_F32, opts=o, ws=ws)
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
        rd = M.moto_min_modes(plan, m1, 4, M.MOTO_F32)  # no options at all
        torch.cuda.synchronize()
        extra["min_modes_128_k4_default_opts"] = {"iters": rd.iters, "status": M.STATUS_NAMES[rd.status],
                                                  "max_iter": M.eig_opts(M.MOTO_F32).max_iter,
                                                  "lambda": [round(float(x), 6) for x in rd.evals.cpu()]}
        extra["min_modes_128_k4_ms"] = round(1e3 * float(np.median(times)), 3)
        extra["min_modes_128_k4_iters"] = r.iters
        extra["min_modes_128_k4_n_hvp"] = int(r.n_hvp)
        extra["min_modes_128_k4_status"] = M.STATUS_NAMES[r.status]
        extra["min_modes_workspace_bytes"] = ws.nbytes
        extra["dense_hessian_bytes_avoided"] = (2 * N) ** 2 * 8
        # block width: guard vectors beyond k trade per-iteration work for iterations
        sweep = {}
        for guard in (() if args.eigen_only else (2, 4, 8)):
            wsg = M.EigWorkspace(plan, M.MOTO_F32, 4, guard)
            og = M.eig_opts(M.MOTO_F32, tol=1e-5, max_iter=400, guard=guard)
            M.moto_min_modes(plan, m1, 4, M.MOTO_F32, opts=og, ws=wsg)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            rg = M.moto_min_modes(plan, m1, 4, M.MOTO_F32, opts=og, ws=wsg)
            torch.cuda.synchronize()
            sweep[f"guard{guard}"] = {"ms": round(1e3 * (time.perf_counter() - t0), 3), "iters": rg.iters,
                                      "status": M.STATUS_NAMES[rg.status]}
        extra["min_modes_128_k4_guard_sweep"] = sweep
        # the second inner solver on the same state: thick-restart Lanczos
        lz = {}
        for mm in (32, 48):
            wsl = M.LanczosWorkspace(plan, M.MOTO_F32, mm)
            ol = M.lanczos_opts(M.MOTO_F32, tol=1e-5, m_max=mm)
            M.moto_min_modes_lanczos(plan, m1, 4, M.MOTO_F32, opts=ol, ws=wsl)
            torch.cuda.synchronize()
            ts = []
            for _ in range(5):
                t0 = time.perf_counter()
                rl = M.moto_min_modes_lanczos(plan, m1, 4, M.MOTO_F32, opts=ol, ws=wsl)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            lz[f"m_max{mm}"] = {"ms": round(1e3 * float(np.median(ts)), 3), "restarts": rl.iters,
                                "n_hvp": int(rl.n_hvp), "status": M.STATUS_NAMES[rl.status],
                                "lambda": [round(float(x), 6) for x in rl.evals.cpu()],
                                "workspace_bytes": wsl.nbytes}
        extra["lanczos_128_k4"] = lz
        extra["lobpcg_128_k4_lambda"] = [round(float(x), 6) for x in r.evals.cpu()]
    c0_gpu = {}
    if not args.hvp_only and not args.eigen_only:
        # the plain method on the 16x16 nearest-neighbour model, FP64: one
        # search per seed to ||F|| < 1e-6 with k = 1, certified with k = 2;
        # R = 3 starts (seeds 0-7) and the R = 1 collapse starts (seeds 0-7)
        print("[bench] 16x16 plain-method searches (FP64)", file=sys.stderr, flush=True)
        p0 = S.ham_nn(16)
        plan0 = M.Plan.from_params(p0)
        so0 = M.search_opts(M.MOTO_F64, tau_F=1e-6, k=1, k_cert=2)
        for tag, R in (("R3", 3.0), ("R1", 1.0)):
            rows = []
            for sd in range(8):
                m0h = S.add_tilt_noise(S.skyrmion(16, 16, R), 0.05, np.random.default_rng(sd))
                md = torch.as_tensor(m0h, device="cuda")
                E0, _, _, _, _ = M.moto_energy_grad(plan0, md, want_grad=False, want_F=False)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                r0, _, _ = M.moto_saddle_search(plan0, md, M.MOTO_F64, opts=so0)
                torch.cuda.synchronize()
                rows.append((time.perf_counter() - t0, r0, float(E0)))
            hist = {}
            for _, r0, _ in rows:
                hist[M.STATUS_NAMES[r0.status]] = hist.get(M.STATUS_NAMES[r0.status], 0) + 1
            c0_gpu[tag] = rows
            extra[f"plain_16x16_{tag}_f64"] = {
                "searches": 8, "median_ms": round(1e3 * float(np.median([t for t, _, _ in rows])), 2),
                "mean_outer_iters": round(float(np.mean([r0.iters for _, r0, _ in rows])), 1),
                "mean_hvp": round(float(np.mean([r0.n_hvp for _, r0, _ in rows])), 1),
                "status": hist,
                "seed0": {"lambda": [rows[0][1].lambda1, rows[0][1].lambda2],
                          "dE": rows[0][1].E - rows[0][2], "iters": rows[0][1].iters}}
        del plan0
    if not args.hvp_only and not args.eigen_only and args.large:
        # tangent HVP at 512x512: one state with the 24-column block of a
        # k = 8 solve (L2/MALL-resident), and 16 states x 4 vectors (335 MB,
        # beyond the 256 MB MALL)
        print("[bench] 512x512 tangent HVP bandwidth", file=sys.stderr, flush=True)
        L2 = 512
        plan5 = M.Plan.from_params(S.ham_3shell(L2))
        h5 = {}
        for tag, nb5, nv5 in (("one_state_24vec", 1, 24), ("batch16_4vec", 16, 4)):
            m5, c5, V5, W5, _ = hvp_inputs(M, S, torch, plan5, L2, nb5, nv5, n_distinct=min(nb5, 4))
            M.moto_tangent_hvp_autotune(plan5, m5, c5, V5, W5, batch=nb5, reps=5)
            _, per5, _ = time_hvp(M, torch, plan5, m5, c5, V5, W5, nb5, 20, 5)
            t5 = float(np.median(per5)) * 1e-3
            b5 = (12 + 16 * nv5) * L2 * L2 * nb5
            h5[tag] = {"ms": round(1e3 * t5, 4), "Gsite_vectors_per_s": round(nb5 * L2 * L2 * nv5 / t5 / 1e9, 2),
                       "GBps_alg": round(b5 / t5 / 1e9, 1), "frac_of_8TBps": round(b5 / t5 / 8e12, 3),
                       "footprint_MB": round((b5 + 4 * L2 * L2 * nb5) / 1e6, 1)}
            del m5, c5, V5, W5
        extra["hvp_512"] = h5
        del plan5
        torch.cuda.empty_cache()
    if not args.hvp_only and not args.eigen_only and args.large:
        # 512x512 with two skyrmions (Q = 2), k = 8: the size where a dense
        # tangent Hessian (2N)^2 FP64 = 2.2 TB is out of reach
        print("[bench] 512x512 two-skyrmion state, k=8 FP32 eigen-solve", file=sys.stderr, flush=True)
        L2 = 512
        p2 = S.ham_3shell(L2)
        plan2 = M.Plan.from_params(p2)
        m2 = torch.as_tensor(S.two_skyrmions(L2), device="cuda")
        o2 = M.eig_opts(M.MOTO_F32, tol=1e-5, max_iter=200)
        ws2 = M.EigWorkspace(plan2, M.MOTO_F32, 8)
        M.moto_min_modes(plan2, m2, 8, M.MOTO_F32, opts=o2, ws=ws2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r2 = M.moto_min_modes(plan2, m2, 8, M.MOTO_F32, opts=o2, ws=ws2)
        torch.cuda.synchronize()
        extra["min_modes_512_two_skyrmions_k8"] = {
            "ms": round(1e3 * (time.perf_counter() - t0), 2), "iters": r2.iters, "n_hvp": int(r2.n_hvp),
            "status": M.STATUS_NAMES[r2.status], "workspace_bytes": ws2.nbytes,
            "dense_hessian_bytes": (2 * L2 * L2) ** 2 * 8,
            "lambda": [round(float(x), 6) for x in r2.evals.cpu()]}
        # the band Lanczos on the same state (depth 64): the magnon band
        # bottom that LOBPCG does not resolve within its cap
        wsl2 = M.LanczosWorkspace(plan2, M.MOTO_F32, 64)
        ol2 = M.lanczos_opts(M.MOTO_F32, tol=1e-5, m_max=64, max_restarts=400)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rl2 = M.moto_min_modes_lanczos(plan2, m2, 8, M.MOTO_F32, opts=ol2, ws=wsl2)
        torch.cuda.synchronize()
        extra["min_modes_512_two_skyrmions_k8_lanczos64"] = {
            "ms": round(1e3 * (time.perf_counter() - t0), 2), "restarts": rl2.iters, "n_hvp": int(rl2.n_hvp),
            "status": M.STATUS_NAMES[rl2.status], "workspace_bytes": wsl2.nbytes,
            "lambda": [round(float(x), 6) for x in rl2.evals.cpu()]}
        del m2, ws2, wsl2
        # time and workspace of the k = 2 solve against the lattice size
        # (the paper's Fig. 2b-c axes), uniform and skyrmion states
        scal = {}
        for Ls in (16, 32, 64, 128, 256, 512, 1024):
            ps = S.ham_3shell(Ls)
            pls = M.Plan.from_params(ps)
            for kind in ("fm", "skyrmion"):
                ms_ = S.uniform(Ls * Ls) if kind == "fm" else S.three_shell_start(Ls, seed=0, kind="skyrmion")
                md_ = torch.as_tensor(ms_, device="cuda")
                os_ = M.eig_opts(M.MOTO_F32, tol=1e-5, max_iter=200)
                wss = M.EigWorkspace(pls, M.MOTO_F32, 2)
                M.moto_min_modes(pls, md_, 2, M.MOTO_F32, opts=os_, ws=wss)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rs_ = M.moto_min_modes(pls, md_, 2, M.MOTO_F32, opts=os_, ws=wss)
                torch.cuda.synchronize()
                scal[f"{Ls}_{kind}"] = {"ms": round(1e3 * (time.perf_counter() - t0), 2), "iters": rs_.iters,
                                        "status": M.STATUS_NAMES[rs_.status], "workspace_MB": round(wss.nbytes / 2**20, 2)}
                del md_, wss
            print(f"[bench]   k=2 solves on {Ls}x{Ls} done", file=sys.stderr, flush=True)
        extra["min_modes_k2_scaling"] = scal
        torch.cuda.empty_cache()
    if not args.hvp_only and not args.eigen_only and args.shells35 > 0:
        # the many-shell regime: the 35-shell Pd/Fe/Ir(111) exchange of Table S1
        # (360 bonds per site) on 128x128 lattices, FP32 frame HVP
        B35 = args.shells35
        print(f"[bench] 35-shell HVP, {B35} x 128x128 x {nvec} FP32 vectors", file=sys.stderr, flush=True)
        p35 = S.ham_pdfeir(L)
        plan35 = M.Plan.from_params(p35)
        spec35 = S.fixed_size_spec(B35, L, seed=35)
        m35 = torch.as_tensor(np.stack([S.batch_member(spec35, i) for i in range(B35)]), device="cuda")
        _, _, c35, _, _ = M.moto_energy_grad(plan35, m35, want_grad=False, want_F=False)
        m35f, c35f = m35.float().contiguous(), c35.float().contiguous()
        g35 = torch.Generator(device="cuda").manual_seed(350)
        V35 = torch.randn(B35, nvec, 2, N, device="cuda", generator=g35)
        W35 = torch.empty_like(V35)
        _, per35, _ = time_hvp(M, torch, plan35, m35f, c35f, V35, W35, B35, 10, 3)
        t35 = float(np.mean(per35)) * 1e-3
        sv = B35 * nvec * N
        n_off = 360
        # per site-vector: one add per bond and component, one multiply per
        # shell and component, DMI (6 bonds x 4) and frame in/out (12)
        ops = n_off * 3 + 35 * 3 + 24 + 12
        lds_bytes = n_off * 3 * 4
        extra["hvp_35shell_128"] = {
            "batch": B35, "n_vec": nvec, "ms_per_launch": round(1e3 * t35, 4),
            "Gsite_vectors_per_s": round(sv / t35 / 1e9, 3),
            "valu_ops_per_site_vector": ops, "valu_Tops": round(sv * ops / t35 / 1e12, 2),
            "valu_frac_of_39.3T": round(sv * ops / t35 / 39.3e12, 3),
            "lds_bytes_per_site_vector": lds_bytes, "lds_TBps": round(sv * lds_bytes / t35 / 1e12, 2),
            "lds_frac_of_78.6TBps": round(sv * lds_bytes / t35 / 78.6e12, 3)}
        del m35, c35, m35f, c35f, V35, W35
        torch.cuda.empty_cache()
    if not args.hvp_only and not args.eigen_only and args.population > 0:
        # explorer scale: the two lowest modes of a population of perturbed
        # 128x128 states, in lock step and one at a time; then the whole
        # objective evaluation (candidates, l1 diversity, charge, gap)
        Pp = args.population
        print(f"[bench] population of {Pp} 128x128 k=2 FP32 eigen-solves", file=sys.stderr, flush=True)
        spec_p = S.fixed_size_spec(Pp, L, seed=2024)
        mp_all = torch.as_tensor(np.stack([S.batch_member(spec_p, i) for i in range(Pp)]), device="cuda")
        op = M.eig_opts(M.MOTO_F32, tol=1e-5, max_iter=400)
        wsp = M.PopulationWorkspace(plan, M.MOTO_F32, Pp, 2)
        M.moto_min_modes_population(plan, mp_all, 2, M.MOTO_F32, opts=op, ws=wsp)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rp = M.moto_min_modes_population(plan, mp_all, 2, M.MOTO_F32, opts=op, ws=wsp)
        torch.cuda.synchronize()
        t_pop = time.perf_counter() - t0
        ws1 = M.EigWorkspace(plan, M.MOTO_F32, 2)
        M.moto_min_modes(plan, mp_all[0].contiguous(), 2, M.MOTO_F32, opts=op, ws=ws1)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its1 = 0
        for i in range(Pp):
            r1 = M.moto_min_modes(plan, mp_all[i].contiguous(), 2, M.MOTO_F32, opts=op, ws=ws1)
            its1 += r1.iters
        torch.cuda.synchronize()
        t_one = time.perf_counter() - t0
        st_hist = {}
        for stt in rp.status:
            st_hist[M.STATUS_NAMES[stt]] = st_hist.get(M.STATUS_NAMES[stt], 0) + 1
        extra["population_eigen_128_k2"] = {
            "P": Pp, "lock_step_ms": round(1e3 * t_pop, 2), "one_at_a_time_ms": round(1e3 * t_one, 2),
            "speedup": round(t_one / t_pop, 2), "max_iters": int(max(rp.iters)),
            "mean_iters": round(float(np.mean(rp.iters)), 1), "one_at_a_time_mean_iters": round(its1 / Pp, 1),
            "status": st_hist}
        print(f"[bench] explorer objectives, population {Pp} on 128x128, masked disc, archive 8", file=sys.stderr,
              flush=True)
        x0e = torch.as_tensor(S.three_shell_start(L, seed=0, kind="skyrmion"), device="cuda")
        rng = np.random.default_rng(24)
        mask_e = torch.as_tensor(S.random_mask_disc(L, L, 20.0), device="cuda")
        de = torch.as_tensor(0.25 * rng.standard_normal((Pp, 3, N)), device="cuda")
        arch = torch.as_tensor(np.stack([S.batch_member(spec_p, i) for i in range(8)]), device="cuda")
        oe = M.explorer_opts(M.MOTO_F32, eig={"tol": 1e-5, "max_iter": 400})
        M.moto_explorer_objectives(plan, x0e, de, M.MOTO_F32, mask=mask_e, archive=arch, opts=oe)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        re_ = M.moto_explorer_objectives(plan, x0e, de, M.MOTO_F32, mask=mask_e, archive=arch, opts=oe)
        torch.cuda.synchronize()
        t_exp = time.perf_counter() - t0
        extra["explorer_128_P%d" % Pp] = {
            "wall_ms": round(1e3 * t_exp, 2), "candidates_per_s": round(Pp / t_exp, 1),
            "max_iters": int(re_.res["iters"].max()),
            "converged": int((re_.res["status"] == M.CONVERGED).sum()),
            "gap_median": float(np.median(re_.res["gap"])), "l1_min_median": float(np.median(re_.res["l1_min"]))}
    if not args.hvp_only and not args.eigen_only:
        # differentiation form on 64x64 (energy, backward, double backward), FP32 spins
        from paper_2509_26269_amd import autograd as AG

        p64 = S.ham_3shell(64)
        m64 = torch.as_tensor(S.random_texture(4096, np.random.default_rng(64)), dtype=torch.float32,
                              device="cuda").requires_grad_(True)
        th = AG.theta_of(p64).requires_grad_(True)
        u = torch.randn(3, 4096, device="cuda", generator=torch.Generator(device="cuda").manual_seed(65))
        ad = {}
        for name in ("forward", "backward", "double_backward"):
            ts = []
            for rep in range(6):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                E = AG.energy(m64, th, 64, 64)
                if name != "forward":
                    g, = torch.autograd.grad(E, m64, create_graph=(name == "double_backward"))
                    if name == "double_backward":
                        torch.autograd.grad((g * u).sum(), (m64, th))
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            ad[name + "_ms"] = round(1e3 * float(np.median(ts[1:])), 3)
        extra["autograd_64x64_f32"] = ad

    if not args.hvp_only and not args.no_search:
        so = M.search_opts(M.MOTO_F32, tau_F=1e-5, k=2, k_cert=2, max_outer=args.max_outer,
                           eig={"tol": 1e-5, "max_iter": 200})
        extra["search_opts"] = {"tau_F": 1e-5, "k": 2, "k_cert": 2, "max_outer": args.max_outer,
                                "eig_tol_rel": 1e-5, "eig_max_iter": 200, "hvp": "f32", "rule": "lbfgs(8)"}

        som = M.search_opts(M.MOTO_F32, tau_F=1e-5, k=2, k_cert=2, max_outer=args.max_outer_masked,
                            eig={"tol": 1e-5, "max_iter": 200})

        def summary(res, el, cap):
            hist = {}
            for r in res:
                hist[M.STATUS_NAMES[r.status]] = hist.get(M.STATUS_NAMES[r.status], 0) + 1
            its = int(sum(r.iters for r in res))
            return {"searches": len(res), "wall_s": round(el, 3),
                    "searches_per_s": round(len(res) / el, 4),
                    "certified_saddles_per_s": round(sum(1 for r in res if r.status == M.SADDLE) / el, 4),
                    "outer_iters_per_s": round(its / el, 1),
                    "mean_outer_iters": round(its / len(res), 1),
                    "max_outer_iters": int(max(r.iters for r in res)),
                    "outer_cap": cap, "ended_at_cap": int(sum(1 for r in res if r.iters >= cap)),
                    "hvp_columns_per_outer": round(sum(r.n_hvp for r in res) / max(its, 1), 1),
                    "status": hist}

        def batched_leg(name, Ls, starts, hp, opts, cap, masks=None, tune=False):
            mall = torch.as_tensor(np.concatenate([x.reshape(-1) for x in starts]), device="cuda")
            mk = None if masks is None else torch.as_tensor(np.concatenate(masks), device="cuda")
            tiles, t_tune = None, 0.0
            if tune:
                t0 = time.perf_counter()
                tiles = M.moto_saddle_search_batched_autotune(hp, list(Ls), mall, opts, mask_all=mk)
                t_tune = time.perf_counter() - t0
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = M.moto_saddle_search_batched(hp, list(Ls), mall, opts, mask_all=mk, tiles=tiles)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            extra[name] = summary(res, el, cap)
            if tune:
                names = {M.TILE_32x8: "32x8", M.TILE_16x16: "16x16", M.TILE_64x4: "64x4"}
                by = {}
                for L_, t_ in zip(Ls, tiles):
                    by.setdefault(names[t_], []).append(int(L_))
                extra[name]["autotune_s"] = round(t_tune, 3)
                extra[name]["tiles_by_side"] = {k_: [min(v_), max(v_), len(v_)] for k_, v_ in by.items()}
            return res

        spec = S.fixed_size_spec(max(args.batched, args.searches), L, seed=128)
        if args.batched > 0:
            # the same starts as searches in lock step over the whole chip
            print(f"[bench] {args.batched} saddle searches on {L}x{L} in lock step (population)", file=sys.stderr,
                  flush=True)
            mpop = torch.as_tensor(np.stack([S.batch_member(spec, i) for i in range(args.batched)]), device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            resp, _, _ = M.moto_saddle_search_population(plan, mpop, M.MOTO_F32, opts=so)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            hist = {}
            for r in resp:
                hist[M.STATUS_NAMES[r.status]] = hist.get(M.STATUS_NAMES[r.status], 0) + 1
            its = int(sum(r.iters for r in resp))
            extra["population_128"] = summary(resp, el, args.max_outer)
            # The same starts with the climb confined to a disc of radius 8
            # around the core (the masked subspace Omega): outside it the
            # texture stays fixed, which pins the two soft translation modes
            # that keep unmasked searches on a 128x128 lattice from meeting
            # the force tolerance.
            print(f"[bench] {args.batched} masked saddle searches on {L}x{L} in lock step (disc radius 8)",
                  file=sys.stderr, flush=True)
            disc = S.random_mask_disc(L, L, 8.0)
            mmask = torch.as_tensor(np.stack([disc] * args.batched), device="cuda")
            mpop = torch.as_tensor(np.stack([S.batch_member(spec, i) for i in range(args.batched)]), device="cuda")
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            resm, _, _ = M.moto_saddle_search_population(plan, mpop, M.MOTO_F32, mask=mmask, opts=som)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            extra["population_128_masked_disc8"] = summary(resm, el, args.max_outer_masked)
            extra["population_128_masked_disc8"]["masked_sites"] = int(disc.sum())
            del mpop, mmask
            nsm = min(args.searches_masked, args.batched)
            if nsm > 0:
                # the first of the same masked starts one at a time through moto_saddle_search
                print(f"[bench] {nsm} masked saddle searches on {L}x{L} one at a time", file=sys.stderr,
                      flush=True)
                dmask = torch.as_tensor(disc, device="cuda")
                r1s = []
                t0 = time.perf_counter()
                for i in range(nsm):
                    md = torch.as_tensor(S.batch_member(spec, i), device="cuda")
                    r1, _, _ = M.moto_saddle_search(plan, md, M.MOTO_F32, mask=dmask, opts=som)
                    r1s.append(r1)
                    print(f"[bench]   search {i}: {M.STATUS_NAMES[r1.status]} iters={r1.iters}", file=sys.stderr,
                          flush=True)
                torch.cuda.synchronize()
                extra["one_at_a_time_128_masked_disc8"] = summary(r1s, time.perf_counter() - t0,
                                                                  args.max_outer_masked)
        if args.ragged > 0:
            rs = S.ragged_batch_spec(256, seed=26269)
            n = min(args.ragged, 256)
            print(f"[bench] {n} saddle searches on uneven 32..96 lattices in one persistent launch",
                  file=sys.stderr, flush=True)
            batched_leg("batched_ragged_32_96", rs.L[:n], [S.batch_member(rs, i) for i in range(n)], p, so,
                        args.max_outer)
            # the same starts with the climb confined to a disc of radius 10
            # around the lattice centre (the textures' cores), tile shapes from
            # the autotuner
            masks = [S.random_mask_disc(Lb, Lb, 10.0).astype(np.uint8) for Lb in rs.L[:n]]
            print(f"[bench] {n} masked saddle searches on uneven lattices, autotuned tiles, one persistent launch",
                  file=sys.stderr, flush=True)
            batched_leg("batched_ragged_32_96_masked_disc10", rs.L[:n], [S.batch_member(rs, i) for i in range(n)], p,
                        som, args.max_outer_masked, masks=masks, tune=True)
            ns1 = min(args.ragged_single, n)
            if ns1 > 0:
                print(f"[bench] {ns1} of them one at a time", file=sys.stderr, flush=True)
                r1s = []
                t0 = time.perf_counter()
                for i in range(ns1):
                    Lb = rs.L[i]
                    pl = M.Plan.from_params(p.with_size(Lb, Lb))
                    md = torch.as_tensor(S.batch_member(rs, i), device="cuda")
                    r1, _, _ = M.moto_saddle_search(pl, md, M.MOTO_F32, mask=torch.as_tensor(masks[i], device="cuda"),
                                                    opts=som)
                    r1s.append(r1)
                torch.cuda.synchronize()
                extra["one_at_a_time_ragged_masked_disc10_first%d" % ns1] = summary(r1s, time.perf_counter() - t0,
                                                                                    args.max_outer_masked)
        def one_at_a_time(name, rule):
            sor = M.search_opts(M.MOTO_F32, tau_F=1e-5, k=2, k_cert=2, max_outer=args.max_outer,
                                eig={"tol": 1e-5, "max_iter": 200}, step={"rule": rule})
            print(f"[bench] {args.searches} saddle searches on {L}x{L} one at a time ({name})", file=sys.stderr,
                  flush=True)
            stats = {}
            t0 = time.perf_counter()
            n_iter = 0
            n_hvp = 0
            for i in range(args.searches):
                md = torch.as_tensor(S.batch_member(spec, i), device="cuda")
                res1, _, _ = M.moto_saddle_search(plan, md, M.MOTO_F32, opts=sor)
                stats[M.STATUS_NAMES[res1.status]] = stats.get(M.STATUS_NAMES[res1.status], 0) + 1
                n_iter += res1.iters
                n_hvp += res1.n_hvp
                print(f"[bench]   search {i}: {M.STATUS_NAMES[res1.status]} iters={res1.iters}", file=sys.stderr,
                      flush=True)
            el = time.perf_counter() - t0
            extra[name] = {"searches": args.searches, "wall_s": round(el, 3),
                           "searches_per_s": round(args.searches / el, 4),
                           "outer_iters_per_s": round(n_iter / el, 1),
                           "mean_outer_iters": round(n_iter / args.searches, 1),
                           "hvp_columns_per_outer": round(n_hvp / max(n_iter, 1), 1),
                           "status": stats}

        if args.searches > 0:
            one_at_a_time("one_at_a_time_128", M.RULE_LBFGS)
            # the paper's second outer optimiser on the same starts
            one_at_a_time("one_at_a_time_128_cg", M.RULE_CG)

    if not args.hvp_only and not args.eigen_only and not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        import oracle as O

        n1, el1 = cpu_baseline(O, S, p, base, nvec, budget_s=8.0)
        print("[bench] CPU oracle baseline on all host cores", file=sys.stderr, flush=True)
        na, ela, ncores, _ = cpu_baseline_all_cores(L, nvec, budget_s=10.0)
        out["cpu_baseline"] = {
            "value": round(na * N / ela / 1e9, 6),
            "unit": "Gsite/s",
            "cores": ncores,
            "kind": "oracle",
            "sample": f"{na} FP64 oracle HVPs ({na // nvec} {L}x{L} states from {len(base)} distinct seeded "
                      f"states, x {nvec} vectors, frame coordinates in and out) in {ela:.1f} s on {ncores} "
                      f"processes (one per core)",
            "value_1core": round(n1 * N / el1 / 1e9, 6),
            "sample_1core": f"{n1} HVPs in {el1:.1f} s on one core",
        }
    if not args.hvp_only and not args.eigen_only and not args.no_cpu:
        import oracle as O

        if c0_gpu:
            # the oracle on seed 0 of each 16x16 start family (host process)
            h0 = O.Ham(**S.ham_nn(16).asdict())
            for tag, R in (("R3", 3.0), ("R1", 1.0)):
                m0h = S.add_tilt_noise(S.skyrmion(16, 16, R), 0.05, np.random.default_rng(0))
                t0 = time.perf_counter()
                ro = O.saddle_search(h0, m0h, tau_F=1e-6, k=1)
                el0 = time.perf_counter() - t0
                rg = c0_gpu[tag][0][1]
                extra[f"plain_16x16_{tag}_f64"]["oracle_seed0"] = {
                    "s": round(el0, 2), "status": int(ro.status), "iters": int(ro.iters),
                    "gpu_status_matches": int(rg.status) == int(ro.status),  # same status codes
                    "dE_gpu_vs_oracle": abs(rg.E - ro.E)}
        if args.batched > 0:
            # the oracle climb on the first starts of the 128x128 search legs,
            # all host cores, 3 outer steps each (a bounded sample)
            print("[bench] CPU oracle searches on 128x128 (all cores, 3 outer steps each)", file=sys.stderr,
                  flush=True)
            its, elc, ncs = cpu_search_all_cores(L, 3)
            extra["oracle_search_128"] = {"outer_iters_per_s": round(its / elc, 3), "cores": ncs,
                                          "sample": f"{ncs} starts x 3 outer steps (+ certification), "
                                                    f"{its} outer steps in {elc:.1f} s"}
    out["extra"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
