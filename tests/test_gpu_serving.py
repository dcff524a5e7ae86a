"""Serving (hm_server): continuous batching of compressions and applies on one
GPU with resident H-matrices and admission by device-memory footprint.

The bar for results: every served request computes exactly what the same
call computes alone (same kernels on the same inputs; nothing depends on what
else runs), checked to 1e-12 relative (normally bit-exact), for FP64 and for
the mixed form."""
import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2205_03406_amd as m
    return m


JOBS = [  # (points, leaf, kernel, tol, r, prec, seed)
    (lambda: workloads.star_curve(3000), 64, "log", 1e-8, 24, 0, 11),
    (lambda: workloads.sphere(2500, 21), 128, "inv_r", 1e-6, 32, 1, 12),
    (lambda: workloads.ellipse(1800, 1.5, 0.6), 64, "log", 1e-6, 24, 1, 13),
    (lambda: workloads.star_curve(5000), 64, "log", 1e-6, 24, 0, 14),
]


def _alone(hm, pts, leaf, kernel, tol, r, prec, seed):
    T = hm.Tree(pts, leaf).color()
    return T, hm.compress(T, T.kernel_blackbox(kernel), tol=tol, r=r, seed=seed, prec=prec)


def _apply(hm, H, X):
    dt = torch.float32 if X.dtype == np.float32 else torch.float64
    Xd = torch.from_numpy(np.ascontiguousarray(X.T)).cuda().t()
    Y = hm.colmajor(X.shape[0], X.shape[1], dtype=dt)
    H.matvec(Xd, Y)
    torch.cuda.synchronize()
    return Y.double().cpu().numpy()


def _drain(srv, want, on_done=None):
    got = {}
    while len(got) < want:
        for c in srv.poll(wait_ms=2000):
            got[c["id"]] = c
            if on_done:
                on_done(c)
    return got


def test_served_results_equal_alone(hm):
    srv = hm.Server(nslots=3)
    pts = [j[0]() for j in JOBS]
    hids = []
    for (mk, leaf, ker, tol, r, prec, seed), p in zip(JOBS, pts):
        hids.append(srv.submit_compress(p, leaf, kernel=ker, tol=tol, r=r, prec=prec, seed=seed))
    # applies queued right behind the compressions (they wait for them), in
    # both precisions, with 1..33 right-hand sides
    rng = np.random.default_rng(5)
    mv = {}
    for k in range(24):
        i = k % len(JOBS)
        dt = np.float32 if k % 2 else np.float64
        X = rng.standard_normal((pts[i].shape[0], 1 + (7 * k) % 33)).astype(dt)
        mv[srv.submit_matvec(hids[i], X)] = (i, X)
    done = _drain(srv, len(JOBS) + len(mv))
    assert all(c["status"] == 0 for c in done.values()), [c for c in done.values() if c["status"]]
    worst = 0.0
    alone = [_alone(hm, p, *j[1:]) for j, p in zip(JOBS, pts)]
    for rid, (i, X) in mv.items():
        want = _apply(hm, alone[i][1], X)
        got = done[rid]["Y"].astype(np.float64)
        d = np.linalg.norm(got - want) / np.linalg.norm(want)
        worst = max(worst, d)
        assert d <= 1e-12, (rid, i, d)
    # the resident H-matrices themselves
    for i, h in enumerate(hids):
        X = rng.standard_normal((pts[i].shape[0], 3))
        a = _apply(hm, srv.hmatrix(h), X)
        b = _apply(hm, alone[i][1], X)
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(b)
    print("served vs alone, worst relative difference:", worst)
    info = srv.info()
    assert info["residents"] == len(JOBS) and info["pending"] == 0 and info["running"] == 0
    srv.close()


def test_applies_overlap_a_running_compression(hm):
    """Continuous batching: applies on a resident H-matrix are admitted and
    finish while a large compression is still running on another slot."""
    srv = hm.Server(nslots=4)
    small = workloads.star_curve(3000)
    h0 = srv.submit_compress(small, 64, tol=1e-8, r=24, seed=1)
    _drain(srv, 1)
    big = srv.submit_compress(workloads.sphere(40000, 7), 128, kernel="inv_r", tol=1e-6, r=32,
                              seed=2)
    rng = np.random.default_rng(1)
    ids = [srv.submit_matvec(h0, rng.standard_normal((3000, 8))) for _ in range(12)]
    done = _drain(srv, 13)
    cb = done[big]
    assert cb["status"] == 0
    inside = [done[i] for i in ids if done[i]["t_end"] < cb["t_end"] and done[i]["t_start"] >= cb["t_admit"]]
    print("compression [%.3f, %.3f] s; applies finished inside it: %d of %d"
          % (cb["t_start"], cb["t_end"], len(inside), len(ids)))
    assert len(inside) >= 1
    srv.close()


def test_admission_by_memory_budget(hm):
    """A budget that holds one compression at a time serializes compressions
    (their device-time intervals do not overlap); a request larger than the
    budget fails with HM_E_NOMEM instead of waiting forever."""
    pts = [workloads.star_curve(4000 + 500 * i) for i in range(3)]
    # footprint of the largest: measured by a first server with a large budget
    probe = hm.Server(nslots=1)
    hp = probe.submit_compress(pts[-1], 64, tol=1e-8, r=24, seed=3)
    fp = _drain(probe, 1)[hp]["bytes"]
    probe.close()
    srv = hm.Server(nslots=3, hbm_budget=int(1.5 * fp), compress_slots=3)
    ids = [srv.submit_compress(p, 64, tol=1e-8, r=24, seed=3) for p in pts]
    # each H-matrix is released when its compression completes, so the
    # budget is taken by work in flight (a second compression never fits)
    done = _drain(srv, 3, on_done=lambda c: srv.release(c["hmatrix"]))
    iv = sorted((done[i]["t_start"], done[i]["t_end"]) for i in ids)
    assert all(c["status"] == 0 for c in done.values())
    for (a0, a1), (b0, b1) in zip(iv, iv[1:]):
        assert b0 >= a1 - 1e-6, iv
    srv.close()
    tiny = hm.Server(nslots=1, hbm_budget=fp // 4)
    rid = tiny.submit_compress(pts[-1], 64, tol=1e-8, r=24, seed=3)
    c = _drain(tiny, 1)[rid]
    assert c["status"] == hm.HM_E_NOMEM
    tiny.close()


def test_release_and_errors(hm):
    srv = hm.Server(nslots=2)
    p = workloads.star_curve(2000)
    h = srv.submit_compress(p, 64, tol=1e-8, r=24, seed=4)
    _drain(srv, 1)
    assert srv.info()["residents"] == 1
    srv.release(h)
    assert srv.info()["residents"] == 0
    with pytest.raises(hm.HMError):
        srv.submit_matvec(h, np.zeros((2000, 1)))
    with pytest.raises(hm.HMError):
        srv.submit_matvec(12345, np.zeros((10, 1)))
    srv.close()


@pytest.mark.parametrize("fmt", ["h1", "h1_mixed", "uniform", "h2"])
def test_request_footprints_cover_their_allocations(hm, fmt):
    """Admission reserves a request's footprint (the completion's `bytes`),
    so that estimate must cover the device memory the request takes.  With a
    counting allocator under the server and one request at a time, the peak
    of the allocator's live bytes while a request runs, above what was live
    before it, stays within the request's bytes: a compression in each format
    (the H-matrix it leaves resident included) and applies of 1 to 300
    right-hand sides in both precisions."""
    kw = dict(h1={}, h1_mixed=dict(prec=hm.HM_PREC_MIXED), uniform=dict(uniform=True),
              h2=dict(h2=True))[fmt]
    al = hm.TorchAllocator()
    srv = hm.Server(nslots=1, allocator=al)
    pts = workloads.sphere(6000, 5)
    base = al.live_bytes()
    al.reset_peak()
    h = srv.submit_compress(pts, 64, kernel="inv_r", tol=1e-6, r=32, seed=9, **kw)
    c = _drain(srv, 1)[h]
    assert c["status"] == 0
    used = al.peak_bytes - base
    print("%s compression: peak %d of a %d byte footprint" % (fmt, used, c["bytes"]))
    assert 0 < used <= c["bytes"], (used, c["bytes"])
    rng = np.random.default_rng(6)
    for nrhs, dt in [(1, np.float64), (16, np.float32), (300, np.float64), (300, np.float32)]:
        base = al.live_bytes()
        al.reset_peak()
        rid = srv.submit_matvec(h, rng.standard_normal((pts.shape[0], nrhs)).astype(dt))
        c = _drain(srv, 1)[rid]
        assert c["status"] == 0
        used = al.peak_bytes - base
        print("  apply %d x %s: peak %.2f MB of %.2f MB" % (nrhs, np.dtype(dt).name, used / 1e6,
                                                          c["bytes"] / 1e6))
        assert 0 < used <= c["bytes"], (nrhs, dt, used, c["bytes"])
    srv.close()
    assert al.live_bytes() == 0
