"""Benchmark: H^1 compression by colored peeling on one GPU.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Headline workload (the largest single-GPU configuration): N = 65536 points
uniform on the unit sphere (normalised Gaussians, seed 3), kernel 1/|x - y|
(diagonal 0), adaptive octree with leaves of at most 128 points, strong
admissibility, relative tolerance 1e-6, p = 10, r = 32 columns per test
matrix, graph-colored test matrices, FP64.  One step = build the tree, color
every graph, compress (all levels and the leaf pass) and apply the result to
one vector.  Inputs are synthetic and seeded; after the host tree they are
resident on the GPU.

The JSON line reports the FP64 path as `value` (GFLOP/s of the algorithmic
work: black box + peel + QR + coupling solves) and beside it the net rate
without the black box, the kernel apply's and the peel's rooflines, the
spectral error (20 power iterations), the mixed FP32/FP64 form, the other
configurations (HODLR line, star curve), the uniform and H^2 formats, products,
the batched form and the served mix.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "peel GFLOP/s + compressions/s at rel err 1e-5 vs plain FP64; p50/p99 ms"
PEAK_FP64_MFMA = 78.6e12
PEAK_FP32_MFMA = 157.3e12
PEAK_HBM = 8.0e12
R_COLS = 24            # star-curve lines (the rank rule: largest rank 8 + p <= 24)
H2_RANK = R_COLS - 10  # fixed rank of the H^2 and fixed-rank uniform lines (r - p)
CPU_SAMPLE_N = 16384   # sphere points of the oracle's timed sample


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=65536, help="headline sphere points")
    ap.add_argument("--sub-steps", type=int, default=10,
                    help="timed steps of each star-curve, HODLR and format sub-line")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-uniform", action="store_true")
    ap.add_argument("--no-product", action="store_true")
    ap.add_argument("--no-h2", action="store_true")
    ap.add_argument("--no-configs", action="store_true", help="skip the HODLR and star-curve lines")
    ap.add_argument("--batched-steps", type=int, default=3)
    ap.add_argument("--no-served", action="store_true")
    ap.add_argument("--served-requests", type=int, default=200)
    ap.add_argument("--served-loads", default="0.8",
                    help="comma-separated offered loads (fractions of the FP64 capacity)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many steps, no extras (for profilers)")
    ap.add_argument("--profile-workload", default="sphere",
                    choices=["sphere", "sphere_mixed", "star", "mixed", "batched", "uniform",
                             "product", "h2"],
                    help="with --profile-steps: which workload the steps run")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="with --profile-steps: add a 1 GiB device copy that calibrates "
                         "the FETCH_SIZE / WRITE_SIZE counters")
    return ap.parse_args()


def step(hm, inst, bb_kernel, x, y, prec, tol, uniform=False, h2=False, rank=0, r=None):
    T = hm.Tree(inst.points, inst.leaf, inst.tree, inst.adm).color()
    bb = T.kernel_blackbox(bb_kernel)
    H = hm.compress(T, bb, rank=rank, tol=0.0 if rank else tol, r=r or inst.r, seed=inst.seed,
                    prec=prec, timing=True, uniform=uniform, h2=h2)
    H.matvec(x, y)
    return T, H


def kapply_traffic_bytes(summary):
    """HBM bytes per kernel-apply launch from a committed counter summary
    (FETCH_SIZE and WRITE_SIZE runs, scaled by the copy calibration), or
    None when the kernel source changed since the counters were taken."""
    import hashlib
    try:
        txt = open(os.path.join(ROOT, "profiles", summary)).read()
        src = open(os.path.join(ROOT, "paper_2205_03406_amd", "csrc", "k_kapply.hip"), "rb").read()
    except OSError:
        return None
    want = hashlib.sha256(src).hexdigest()[:16]
    val = h = None
    for line in txt.splitlines():
        if line.startswith("kapply traffic bytes per launch:"):
            val = float(line.split(":")[1])
        if line.startswith("kapply source sha256 (first 16 hex):"):
            h = line.split(":")[1].strip()
    return val if (val is not None and h == want) else None


def _progress(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def algorithmic_flops(st):
    return st["flops_blackbox"] + st["flops_peel"] + st["flops_qr"] + st["flops_solve"]


def net_flops(st):
    return st["flops_peel"] + st["flops_qr"] + st["flops_solve"]


def run_path(hm, torch, inst, prec, tol, steps, warmup, x, y, uniform=False, h2=False, rank=0,
             r=None):
    """warmup + steps timed steps of one workload; accumulates the stage
    statistics of the timed steps."""
    for _ in range(warmup):
        step(hm, inst, inst.kernel, x, y, prec, tol, uniform, h2, rank, r)
    torch.cuda.synchronize()
    acc = dict(flops=0.0, bb_ms=0.0, bb_flops=0.0, net_flops=0.0, net_ms=0.0, peel_ms=0.0,
               peel_flops=0.0, peel_bytes=0.0, launches=0)
    times = []
    H = T = st = None
    t_all0 = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        T, H = step(hm, inst, inst.kernel, x, y, prec, tol, uniform, h2, rank, r)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        st = H.stats()
        acc["flops"] += algorithmic_flops(st)
        acc["bb_ms"] += st["ms_blackbox"]
        acc["bb_flops"] += st["flops_blackbox"]
        acc["net_flops"] += net_flops(st)
        acc["net_ms"] += st["ms_peel"] + st["ms_qr"] + st["ms_solve"]
        acc["peel_ms"] += st["ms_peel"]
        acc["peel_flops"] += st["flops_peel"]
        acc["peel_bytes"] += st["bytes_peel"]
        # one black-box launch per sampled level (two in the uniform format)
        # and the leaf pass
        acc["launches"] += (2 if uniform or h2 else 1) * sum(1 for c in st["colors"] if c) + 1
    total = time.perf_counter() - t_all0
    return dict(times=times, total=total, H=H, T=T, stats=st, **acc)


def line_of(run, steps, n):
    """Throughput, latency and statistics of one run_path result."""
    st = run["stats"]
    lat = np.array(run["times"]) * 1e3
    return {
        "value": round(run["flops"] / run["total"] / 1e9, 2), "unit": "GFLOP/s",
        "compressions_per_s": round(steps / run["total"], 3),
        "ms_per_step": round(1e3 * run["total"] / steps, 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "net_gflops": round(run["net_flops"] / (run["net_ms"] / 1e3) / 1e9, 2)
        if run["net_ms"] > 0 else None,
        "kapply_tflops": round(run["bb_flops"] / (run["bb_ms"] / 1e3) / 1e12, 3)
        if run["bb_ms"] > 0 else None,
        "colors_per_level": [c for c in st["colors"] if c],
        "leaf_colors": st["leaf_colors"],
        "cols_A": st["cols_A"], "cols_At": st["cols_At"],
        "max_rank": st["max_rank"], "saturated": st["saturated"],
        "floats_per_dof": round(st["nfloats"] / n, 2),
        "device_mb": round(st["device_bytes"] / 2**20, 1),
        "stage_ms": {k: round(st[k], 3) for k in ("ms_blackbox", "ms_peel", "ms_qr", "ms_solve",
                                                  "ms_other", "ms_total")},
    }


def peel_roofline(run, prec_bytes):
    """Achieved rate of the peel stage (the level-truncated products
    subtracted, lr_project / lr_reduce / lr_expand and the finiteness check),
    timed by HIP events around the stage on the compression stream: its
    algorithmic bytes against HBM and its flops against the matrix cores."""
    if run["peel_ms"] <= 0:
        return None
    sec = run["peel_ms"] / 1e3
    gbs = run["peel_bytes"] / sec
    fl = run["peel_flops"] / sec
    peak = PEAK_FP64_MFMA if prec_bytes == 8 else PEAK_FP32_MFMA
    ai = run["peel_flops"] / run["peel_bytes"]
    # the bound is the one the algorithmic intensity selects (ridge = peak
    # flops / HBM bandwidth); both fractions are reported
    mfma = ai >= peak / PEAK_HBM
    return {"kernels": "lr_project_kernel, lr_reduce_kernel, lr_expand_kernel",
            "bound": "mfma" if mfma else "hbm",
            "achieved": round(fl / 1e12, 3) if mfma else round(gbs / 1e9, 1),
            "peak": peak / 1e12 if mfma else PEAK_HBM / 1e9,
            "unit": "TFLOP/s" if mfma else "GB/s",
            "frac": round(fl / peak if mfma else gbs / PEAK_HBM, 4),
            "hbm_gbs": round(gbs / 1e9, 1), "hbm_frac": round(gbs / PEAK_HBM, 4),
            "flops_tflops": round(fl / 1e12, 3), "flops_frac": round(fl / peak, 4),
            "intensity_flop_per_byte": round(ai, 2),
            "algorithmic_bytes_per_compression": run["peel_bytes"] / max(1, len(run["times"])),
            "ms_per_compression": round(run["peel_ms"] / max(1, len(run["times"])), 3)}


def device_errors(hm, torch, T, H, kernel, dtype=None, nprobe=16, iters=20, seed=12):
    """Errors of H against the kernel matrix A, both applied on the device
    (A by the library's FP64 kernel apply, generated on the fly): the probe
    estimate ||(A - H) G||_F / ||A G||_F over nprobe Gaussian vectors, and
    the spectral ratio ||A - H||_2 / ||A||_2 from `iters` power iterations
    on (A - H)* (A - H) and on A* A (A is symmetric for both kernels; H* by
    the adjoint apply)."""
    n = T.n
    rng = np.random.default_rng(seed)

    def dev(M):
        t = hm.colmajor(n, M.shape[1])
        t.copy_(torch.from_numpy(M))
        return t

    def Aop(X):
        Y = hm.colmajor(n, X.shape[1])
        T.kernel_apply(kernel, X, Y, order=hm.HM_ORDER_ORIGINAL)
        return Y

    def Hop(X, trans=False):
        Y = hm.colmajor(n, X.shape[1])
        H.matvec(X, Y, trans=trans)
        return Y

    G = dev(rng.standard_normal((n, nprobe)))
    AG = Aop(G)
    probe = float(torch.linalg.norm(AG - Hop(G)) / torch.linalg.norm(AG))

    def power(op, opT):
        v = dev(rng.standard_normal((n, 1)))
        v /= torch.linalg.norm(v)
        s = 0.0
        for _ in range(iters):
            u = opT(op(v))
            s = float(torch.linalg.norm(u))
            if s == 0.0:
                return 0.0
            v = u / s
        return s ** 0.5

    sd = power(lambda v: Aop(v) - Hop(v), lambda w: Aop(w) - Hop(w, True))
    sa = power(Aop, Aop)
    torch.cuda.synchronize()
    return {"probe_rel_fro": probe, "spectral_rel_power20": sd / sa}


def run_product(hm, torch, inst, H, steps, warmup):
    """Compression of the product H H of the headline compressed operator
    with itself, given only through its applies (two H-matrix applies per
    black-box call): the black box is fast, so peel, QR and couplings carry
    the time.  One step = one compression on the existing tree."""
    T = H.tree
    bh = H.blackbox(hm.HM_ORDER_TREE)
    P = hm.product_blackbox(bh, bh)

    def once():
        return hm.compress(T, P, tol=inst.tol, r=R_COLS, seed=inst.seed + 1, timing=True)

    for _ in range(warmup):
        once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    net_flops = net_ms = bb_ms = 0.0
    for _ in range(steps):
        HP = once()
        st = HP.stats()
        net_flops += st["flops_peel"] + st["flops_qr"] + st["flops_solve"]
        net_ms += st["ms_total"] - st["ms_blackbox"]
        bb_ms += st["ms_blackbox"]
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    n = T.n
    X = hm.colmajor(n, 4)
    X.copy_(torch.from_numpy(np.random.default_rng(8).standard_normal((n, 4))))
    Y, Z, W = hm.colmajor(n, 4), hm.colmajor(n, 4), hm.colmajor(n, 4)
    HP.matvec(X, Y)
    H.matvec(X, Z)
    H.matvec(Z, W)
    torch.cuda.synchronize()
    err = float(torch.linalg.norm(Y - W) / torch.linalg.norm(W))
    return {"workload": "product_of_star_curve_operator_with_itself_N%d_tol%g_r%d"
                        % (n, inst.tol, R_COLS),
            "compressions_per_s": round(steps / total, 3),
            "ms_per_step": round(1e3 * total / steps, 3),
            "blackbox_share": round(bb_ms / (bb_ms + net_ms), 3),
            "net_gflops": round(net_flops / (net_ms / 1e3) / 1e9, 2),
            "max_rank": st["max_rank"], "saturated": st["saturated"],
            "floats_per_dof": round(st["nfloats"] / n, 2),
            "rel_err_vs_applied_product": err,
            "stage_ms": {k: round(st[k], 3) for k in ("ms_blackbox", "ms_peel", "ms_qr",
                                                      "ms_solve", "ms_other", "ms_total")}}


def batched_step(hm, insts, prec):
    F = hm.Tree([i.points for i in insts], insts[0].leaf, insts[0].tree, insts[0].adm).color()
    H = hm.compress(F, F.kernel_blackbox(insts[0].kernel), tol=insts[0].tol, r=insts[0].r,
                    seed=insts[0].seed, prec=prec, timing=True)
    return F, H


def run_batched(hm, torch, steps):
    """64 independent ellipse problems (N log-uniform in [2048, 32768]) as one
    forest: FP32 bulk + FP64 QR, tol 1e-6.  One step = build the 64 trees,
    merge, color, compress; `value` counts each instance's own algorithmic
    work."""
    import workloads
    insts = workloads.batched_ellipses()
    ntot = sum(i.points.shape[0] for i in insts)
    batched_step(hm, insts, hm.HM_PREC_MIXED)          # warm-up
    torch.cuda.synchronize()
    times, flops, bb_ms, bb_flops = [], 0.0, 0.0, 0.0
    t_all = time.perf_counter()
    for _ in range(steps):
        t0 = time.perf_counter()
        F, H = batched_step(hm, insts, hm.HM_PREC_MIXED)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        st = H.stats()
        flops += algorithmic_flops(st)
        bb_ms += st["ms_blackbox"]
        bb_flops += st["flops_blackbox"]
    total = time.perf_counter() - t_all
    # error of the mixed result against the FP64 compression of the forest
    F64, H64 = batched_step(hm, insts, hm.HM_PREC_F64)
    X = hm.colmajor(ntot, 2)
    X.copy_(torch.from_numpy(np.random.default_rng(8).standard_normal((ntot, 2))))
    Y32, Y64 = hm.colmajor(ntot, 2), hm.colmajor(ntot, 2)
    H.matvec(X, Y32)
    H64.matvec(X, Y64)
    torch.cuda.synchronize()
    a, b = Y64.cpu().numpy(), Y32.cpu().numpy()
    lat = np.array(times) * 1e3
    ach = bb_flops / (bb_ms / 1e3)
    # the same forest compressed again and again through a plan: the device
    # pipeline captured once into a HIP graph and replayed (trees, colors and
    # planning are done once, outside the timed replays)
    F = hm.Tree([i.points for i in insts], insts[0].leaf, insts[0].tree, insts[0].adm).color()
    plan = hm.Plan(F, F.kernel_blackbox(insts[0].kernel), tol=insts[0].tol, r=insts[0].r,
                   seed=insts[0].seed, prec=hm.HM_PREC_MIXED)
    plan.execute()
    torch.cuda.synchronize()
    t_rep = time.perf_counter()
    for _ in range(steps):
        plan.execute()
    torch.cuda.synchronize()
    t_rep = (time.perf_counter() - t_rep) / steps
    Yr = hm.colmajor(ntot, 2)
    plan.hmatrix().matvec(X, Yr)
    torch.cuda.synchronize()
    replay_equal = bool(np.array_equal(Yr.cpu().numpy(), b))
    res = {
        "workload": "64_ellipses_log_N2048-32768_leaf64_strong_tol1e-6_r%d_mixed" % insts[0].r,
        "instances": len(insts), "points": ntot, "steps": steps,
        "value": round(flops / total / 1e9, 2), "unit": "GFLOP/s",
        "compressions_per_s": round(len(insts) * steps / total, 3),
        "ms_per_step": round(1e3 * total / steps, 3),
        "p50_ms": round(float(np.percentile(lat, 50)), 3),
        "p99_ms": round(float(np.percentile(lat, 99)), 3),
        "rel_err_vs_fp64": float(np.linalg.norm(a - b) / np.linalg.norm(a)),
        "max_rank": st["max_rank"], "saturated": st["saturated"],
        "graph_replay": {"ms_per_compression_of_all_64": round(1e3 * t_rep, 3),
                         "compressions_per_s": round(len(insts) / t_rep, 3),
                         "graph_nodes": plan.graph_nodes,
                         "equal_to_eager": replay_equal},
        "stage_ms": {k: round(st[k], 3) for k in ("ms_blackbox", "ms_peel", "ms_qr", "ms_solve",
                                                  "ms_other", "ms_total")},
        "kapply": {"kernel": "kapply_kernel<float> (forest items)", "bound": "mfma",
                   "achieved": round(ach / 1e12, 3), "peak": PEAK_FP32_MFMA / 1e12,
                   "unit": "TFLOP/s", "frac": round(ach / PEAK_FP32_MFMA, 4)},
    }
    return res


# ---------------------------------------------------------------- serving
SERVE_RESIDENTS = [("curve", 4096), ("curve", 8192), ("curve", 16384), ("curve", 32768),
                   ("sphere", 4096), ("sphere", 8192), ("sphere", 16384), ("sphere", 32768)]


def _serve_points(geom, n, seed):
    import workloads
    return workloads.star_curve(n) if geom == "curve" else workloads.sphere(n, seed)


def _submit_compress(srv, hm, geom, n, seed, prec):
    pts = _serve_points(geom, n, seed)
    if geom == "curve":
        return srv.submit_compress(pts, 64, kernel="log", tol=1e-6, r=24, prec=prec, seed=seed)
    return srv.submit_compress(pts, 128, kernel="inv_r", tol=1e-6, r=32, prec=prec, seed=seed)


def _serve_once(hm, trace, xs, mixed, nslots, rate_scale):
    """Replay `trace` (arrival times scaled by rate_scale; 0 = all at once) on
    a fresh server holding the 8 resident H-matrices; returns per-request
    latencies (s) by class and the makespan."""
    prec = hm.HM_PREC_MIXED if mixed else hm.HM_PREC_F64
    srv = hm.Server(nslots=nslots)
    res = [_submit_compress(srv, hm, g, n, 900 + i, prec) for i, (g, n) in enumerate(SERVE_RESIDENTS)]
    got = 0
    while got < len(res):
        got += len(srv.poll(wait_ms=1000))
    kinds, due_of, lat = {}, {}, {"compress": [], "matvec": []}
    # latencies from each request's scheduled arrival (a submission that the
    # loop makes late still counts from its arrival); matvec latency split:
    # waiting (arrival -> start on the device stream: submission,
    # admission, a free worker, memory) and running (start -> end: staging,
    # the apply and the copies back, sharing the device with the rest), and
    # of the running time the part between the first copy's start and the
    # last copy's end on the device stream (device events) and the host
    # time spent enqueueing
    split = {"wait": [], "run": [], "enqueue": [], "device": []}
    pending = 0
    t0 = srv.info()["now"]
    i = 0
    fails = 0

    def collect(wait_ms):
        nonlocal pending, fails
        for c in srv.poll(wait_ms=wait_ms):
            k = kinds.pop(c["id"])
            t_arr = due_of.pop(c["id"])
            if c["status"] != 0:
                fails += 1
            lat[k].append(c["t_end"] - t_arr)
            if k == "compress":
                srv.release(c["hmatrix"])
            else:
                split["wait"].append(c["t_start"] - t_arr)
                split["run"].append(c["t_end"] - c["t_start"])
                split["enqueue"].append(c["enqueue_ms"] * 1e-3)
                split["device"].append(c["device_ms"] * 1e-3)
            pending -= 1

    while i < len(trace):
        due = t0 + trace[i].t_arrival * rate_scale
        now = srv.info()["now"]
        if now < due:
            collect(int(min(50.0, (due - now) * 1e3)) if pending else 0)
            if not pending:
                time.sleep(max(0.0, min(0.05, due - srv.info()["now"])))
            continue
        q = trace[i]
        if q.kind == "compress":
            rid = _submit_compress(srv, hm, q.geometry, q.n, q.seed, prec)
        else:
            rid = srv.submit_matvec(res[q.target], xs[mixed][q.target][:q.nrhs].T)
        kinds[rid] = q.kind
        due_of[rid] = due
        pending += 1
        i += 1
    while pending:
        collect(1000)
    t_end = srv.info()["now"]
    srv.close()
    return lat, t_end - t0, fails, split


def run_served(hm, count, loads):
    """Served mix: Poisson arrivals, 1 in 10 a compression (star curve or
    sphere, N log-uniform in [4096, 65536], tol 1e-6), the rest applies with
    1..64 right-hand sides on one of 8 resident H-matrices.  Baseline: the
    plain FP64 path, one request at a time in arrival order (one slot).
    Served: the mixed form with FP32 right-hand sides, 4 slots, admission by
    device memory.  The arrival rate is the given fraction of the FP64
    path's capacity (requests/s it completes back to back)."""
    import workloads
    trace = workloads.serve_trace(count, 1.0, seed=5, n_resident=len(SERVE_RESIDENTS))
    # right-hand sides: one (n, 64) block per resident, sliced per request
    rng = np.random.default_rng(7)
    pool = [rng.standard_normal((64, n)) for _, n in SERVE_RESIDENTS]  # column-major (n, 64)
    xs = {False: pool, True: [x.astype(np.float32) for x in pool]}
    # one back-to-back pass of each form settles the kernel-apply autotuner
    # on the trace's shapes (no timed run pays first-use tuning); then the
    # capacity of the FP64 path: the whole trace back to back on one slot
    _, span, _, _ = _serve_once(hm, trace, xs, False, 1, 0.0)
    _progress("served mix: FP64 warm-up pass %.1f s" % span)
    _, span, _, _ = _serve_once(hm, trace, xs, True, 4, 0.0)
    _progress("served mix: mixed warm-up pass %.1f s" % span)
    _, makespan, _, _ = _serve_once(hm, trace, xs, False, 1, 0.0)
    capacity = count / makespan
    _progress("served mix: FP64 back-to-back pass %.1f s (%.2f requests/s)" % (makespan, capacity))
    out = {"requests": count, "compress_share": round(sum(q.kind == "compress" for q in trace) / count, 3),
           "fp64_capacity_req_per_s": round(capacity, 3), "loads": {}}

    def summary(lat, span, fails, split):
        allv = np.array(lat["compress"] + lat["matvec"]) * 1e3
        d = {"throughput_req_per_s": round(count / span, 3), "failed": fails,
             "p50_ms": round(float(np.percentile(allv, 50)), 3),
             "p99_ms": round(float(np.percentile(allv, 99)), 3)}
        for k in ("compress", "matvec"):
            v = np.array(lat[k]) * 1e3
            d[k] = {"n": len(v), "p50_ms": round(float(np.percentile(v, 50)), 3),
                    "p99_ms": round(float(np.percentile(v, 99)), 3)}
        for k in ("wait", "run", "enqueue", "device"):
            v = np.array(split[k]) * 1e3
            d["matvec"][k + "_p50_ms"] = round(float(np.percentile(v, 50)), 3)
            d["matvec"][k + "_p99_ms"] = round(float(np.percentile(v, 99)), 3)
        return d

    for load in loads:
        rate = load * capacity
        scale = 1.0 / rate  # the trace was drawn at 1 request/s
        base = summary(*_serve_once(hm, trace, xs, False, 1, scale))
        _progress("served mix: load %.2f FP64 one-at-a-time done" % load)
        served = summary(*_serve_once(hm, trace, xs, True, 4, scale))
        _progress("served mix: load %.2f served done" % load)
        out["loads"][str(load)] = {"rate_req_per_s": round(rate, 3), "fp64_fifo": base,
                                   "served_mixed_4slots": served}
    return out


def oracle_threads():
    try:
        from threadpoolctl import threadpool_info
        return max(int(i.get("num_threads", 1)) for i in threadpool_info())
    except Exception:
        return int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2205_03406_amd as hm
    import workloads

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    inst = workloads.config(2, n=args.n)          # sphere, 1/r, tol 1e-6, r = 32
    star = workloads.config(1)                    # star curve, log, tol 1e-8, r = 24

    def vecs(m):
        a = hm.colmajor(m, 1)
        a.copy_(torch.from_numpy(np.random.default_rng(0).standard_normal((m, 1))))
        return a, hm.colmajor(m, 1)

    n = inst.points.shape[0]
    x, y = vecs(n)
    ns = star.points.shape[0]
    xs, ys = vecs(ns)

    if args.profile_steps:
        w = args.profile_workload
        if w == "batched":
            insts = workloads.batched_ellipses()
            for _ in range(args.profile_steps):
                batched_step(hm, insts, hm.HM_PREC_MIXED)
        elif w == "product":
            _, H = step(hm, star, star.kernel, xs, ys, hm.HM_PREC_F64, star.tol)
            run_product(hm, torch, star, H, args.profile_steps, 0)
        elif w in ("sphere", "sphere_mixed"):
            prec = hm.HM_PREC_MIXED if w == "sphere_mixed" else hm.HM_PREC_F64
            for _ in range(args.profile_steps):
                step(hm, inst, inst.kernel, x, y, prec, inst.tol)
        else:
            prec = hm.HM_PREC_MIXED if w == "mixed" else hm.HM_PREC_F64
            tol = 1e-6 if w == "mixed" else star.tol
            for _ in range(args.profile_steps):
                step(hm, star, star.kernel, xs, ys, prec, tol, uniform=w == "uniform",
                     h2=w == "h2", rank=H2_RANK if w in ("h2", "uniform") else 0)
        torch.cuda.synchronize()
        if args.pmc_probe:
            # calibration for the HBM byte counters: one plain device copy of
            # 1 GiB (reads 1 GiB, writes 1 GiB)
            src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
            dst = torch.empty_like(src)
            torch.cuda.synchronize()
            dst.copy_(src)
            torch.cuda.synchronize()
        print("profile run done", flush=True)
        return

    # ---------------- headline: the sphere, FP64
    r64 = run_path(hm, torch, inst, hm.HM_PREC_F64, inst.tol, args.steps, args.warmup, x, y)
    _progress("headline FP64 path done")
    line = line_of(r64, args.steps, n)
    out = {
        "metric": METRIC,
        "value": line.pop("value"),
        "unit": line.pop("unit"),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": line.pop("ms_per_step"),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "sphere_inv_r_N%d_leaf128_adaptive_octree_strong_tol1e-6_r%d"
                               % (n, inst.r),
                   "step": "build_tree+color+compress+hmatvec(1 rhs)"},
    }
    out.update(line)
    # dominant kernel: the on-the-fly kernel apply (FP64 MFMA), timed by HIP
    # events recorded around its launches on the compression stream
    ach = r64["bb_flops"] / (r64["bb_ms"] / 1e3)
    out["roofline"] = {"kernel": "kapply_kernel<double> (1/r)", "bound": "mfma",
                       "achieved": round(ach / 1e12, 3), "peak": PEAK_FP64_MFMA / 1e12,
                       "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_MFMA, 4),
                       "traffic": kapply_traffic_bytes("kapply_f64_sphere_N65536_pmc.md"),
                       "avg_launch_ms": round(r64["bb_ms"] / r64["launches"], 4),
                       "flops_per_launch": r64["bb_flops"] / r64["launches"]}
    out["peel_roofline"] = peel_roofline(r64, 8)
    H = r64["H"]
    out["error_vs_kernel"] = device_errors(hm, torch, r64["T"], H, inst.kernel)
    _progress("headline errors done")

    if not args.no_mixed:
        rmx = run_path(hm, torch, inst, hm.HM_PREC_MIXED, inst.tol, args.steps, args.warmup, x, y)
        G = hm.colmajor(n, 4)
        G.copy_(torch.from_numpy(np.random.default_rng(5).standard_normal((n, 4))))
        Y64, Ymx = hm.colmajor(n, 4), hm.colmajor(n, 4)
        H.matvec(G, Y64)
        rmx["H"].matvec(G, Ymx)
        torch.cuda.synchronize()
        mline = line_of(rmx, args.steps, n)
        mline["tol"] = inst.tol
        mline["rel_err_vs_fp64"] = float(torch.linalg.norm(Ymx - Y64) / torch.linalg.norm(Y64))
        mline["error_vs_kernel"] = device_errors(hm, torch, rmx["T"], rmx["H"], inst.kernel)
        mline["peel_roofline"] = peel_roofline(rmx, 4)
        out["mixed"] = mline
        del rmx
        _progress("headline mixed path done")
    del r64

    # ---------------- the other single-compression configurations
    Hstar = None
    if not args.no_configs:
        hod = workloads.config(0)
        xh, yh = vecs(hod.points.shape[0])
        rh = run_path(hm, torch, hod, hm.HM_PREC_F64, 0.0, args.sub_steps, 2, xh, yh, rank=hod.rank)
        hl = line_of(rh, args.sub_steps, hod.points.shape[0])
        hl["workload"] = "hodlr_line_log_N1024_index_binary_leaf64_weak_k20_r30"
        hl["error_vs_kernel"] = device_errors(hm, torch, rh["T"], rh["H"], hod.kernel)
        out["hodlr"] = hl
        del rh
        rs = run_path(hm, torch, star, hm.HM_PREC_F64, star.tol, args.sub_steps, 2, xs, ys)
        sl = line_of(rs, args.sub_steps, ns)
        sl["workload"] = "star_curve_log_N16384_leaf64_strong_tol1e-8_r%d" % R_COLS
        sl["error_vs_kernel"] = device_errors(hm, torch, rs["T"], rs["H"], star.kernel)
        sl["peel_roofline"] = peel_roofline(rs, 8)
        Hstar = rs["H"]
        rsm = run_path(hm, torch, star, hm.HM_PREC_MIXED, 1e-6, args.sub_steps, 2, xs, ys)
        G = hm.colmajor(ns, 4)
        G.copy_(torch.from_numpy(np.random.default_rng(5).standard_normal((ns, 4))))
        Y64, Ymx = hm.colmajor(ns, 4), hm.colmajor(ns, 4)
        Hstar.matvec(G, Y64)
        rsm["H"].matvec(G, Ymx)
        torch.cuda.synchronize()
        sml = line_of(rsm, args.sub_steps, ns)
        sml["tol"] = 1e-6
        sml["rel_err_vs_fp64"] = float(torch.linalg.norm(Ymx - Y64) / torch.linalg.norm(Y64))
        sl["mixed"] = sml
        out["star_curve"] = sl
        del rsm
        _progress("HODLR and star-curve lines done")

    # ---------------- the paper's other formats on the star curve
    for name, skip, kw in (("uniform", args.no_uniform, dict(uniform=True, rank=H2_RANK)),
                           ("uniform_tol", args.no_uniform, dict(uniform=True)),
                           ("h2", args.no_h2, dict(h2=True, rank=H2_RANK))):
        if skip:
            continue
        run = run_path(hm, torch, star, hm.HM_PREC_F64, star.tol, args.sub_steps, 2, xs, ys, **kw)
        fl = line_of(run, args.sub_steps, ns)
        fl["rank"] = kw.get("rank", 0)
        fl["tol"] = 0.0 if kw.get("rank") else star.tol
        fl["stage1_colors_per_level"] = [c for c in run["stats"]["ucolors"] if c]
        fl["error_vs_kernel"] = device_errors(hm, torch, run["T"], run["H"], star.kernel)
        out[name] = fl
        del run
        _progress(name + " done")

    if not args.no_product and Hstar is not None:
        out["product"] = run_product(hm, torch, star, Hstar, args.sub_steps, 2)
        _progress("product done")

    if not args.no_batched:
        out["batched"] = run_batched(hm, torch, args.batched_steps)
        _progress("batched done")

    if not args.no_served:
        out["served"] = run_served(hm, args.served_requests,
                                   [float(v) for v in args.served_loads.split(",")])

    if not args.no_cpu_baseline:
        # the oracle, untuned, on a bounded sample of the headline workload:
        # the same sphere generator, kernel, leaf, tolerance and r at
        # CPU_SAMPLE_N points; its algorithmic flops are those the GPU counts
        # for a compression of the same sample (same tree, colors and r;
        # ranks agree up to threshold ties)
        import oracle as O
        samp = workloads.config(2, n=CPU_SAMPLE_N)
        xc, yc = vecs(CPU_SAMPLE_N)
        _, Hs = step(hm, samp, samp.kernel, xc, yc, hm.HM_PREC_F64, samp.tol)
        fl = algorithmic_flops(Hs.stats())
        t0 = time.perf_counter()
        OT = O.OTree(samp.points, samp.leaf, samp.tree, samp.adm)
        obb = O.KernelBlackBox(samp.points, samp.kernel)
        O.compress(OT, obb, samp.r, tol=samp.tol, seed=samp.seed)
        tcpu = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": round(fl / tcpu / 1e9, 3), "unit": "GFLOP/s",
                               "cores": oracle_threads(), "kind": "oracle",
                               "sample": "one full oracle compression (tree, colors, dense FP64 "
                                         "black box, recovery) of the headline sphere workload "
                                         "at N=%d, %.1f s" % (CPU_SAMPLE_N, tcpu)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
