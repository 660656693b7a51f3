"""The request server (continuous batching): every request's sinograms are
the same alone (sse_simulate) and in a mix with other requests of different
phantoms and budgets; admission respects the HBM budget; cancellation and
draining work."""
import sys
import time

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2509_05047_amd as sse  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tiny_ctx():
    w = W.WORKLOADS["tiny"]
    ctx = sse.Context(w.scanner, w.sino, w.physics)
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    ctx.load_lut(ld, lut)
    pids = []
    pd, mu, act = W.tiny_cylinder()
    pids.append(ctx.load_phantom(pd, mu, act))
    pd, mu, act = W.uniform_box(n=(10, 12, 8), voxel_mm=(9.0, 8.0, 11.0))
    pids.append(ctx.load_phantom(pd, mu, act))
    pd, mu, act = W.point_source((20.0, -10.0, 5.0), mu=0.0)
    pids.append(ctx.load_phantom(pd, mu, act))
    return ctx, pids


def alone(ctx, pid, n, seed, h_offset=0):
    out = ctx.new_outputs(stats=False)
    ctx.simulate(pid, n, seed, out, h_offset=h_offset)
    torch.cuda.synchronize()
    return out["scatter_counts"].clone(), out["scatter_weights"].clone()


def fetch(ctx, c):
    counts = sse.copy_device_to_tensor(c["scatter_counts"], ctx.n_bins, torch.int32)
    weights = sse.copy_device_to_tensor(c["scatter_weights"], ctx.n_bins, torch.float64)
    return counts, weights


def drain(srv, want, on_done, timeout_s=120.0):
    got = {}
    t0 = time.time()
    while len(got) < want:
        for c in srv.poll(wait_ms=200):
            got[c["id"]] = c
            on_done(c)
        assert time.time() - t0 < timeout_s, "server did not complete in time"
    return got


def same(a, b):
    ca, wa = a
    cb, wb = b
    assert torch.equal(ca, cb)
    nz = wa != 0
    assert torch.equal(nz, wb != 0)
    if nz.any():
        assert float(((wa[nz] - wb[nz]).abs() / wa[nz]).max()) < 1e-12


def test_requests_are_the_same_alone_and_in_the_mix():
    ctx, pids = tiny_ctx()
    # The first request fills the first two ticks (two are kept in flight);
    # the small ones, submitted meanwhile, then share the next tick with it,
    # whatever the kernel's speed.
    reqs = [(pids[0], 20_000_000, 11, 0), (pids[1], 170_000, 12, 0), (pids[2], 90_000, 13, 0),
            (pids[0], 40_000, 14, 1_000_000), (pids[1], 1, 15, 7)]
    ref = [alone(ctx, *r) for r in reqs]
    srv = sse.Server(ctx, max_active=4, tick_histories=5_000_000, chunk_histories=4096)
    own_c = torch.full((ctx.n_bins,), 7, dtype=torch.int32, device="cuda")   # caller-owned, not zeroed by us
    own_w = torch.full((ctx.n_bins,), 3.0, dtype=torch.float64, device="cuda")
    ids = []
    for i, (pid, n, seed, h0) in enumerate(reqs):
        if i == 1:
            ids.append(srv.submit(pid, n, seed, h_offset=h0, counts=own_c, weights=own_w))
        else:
            ids.append(srv.submit(pid, n, seed, h_offset=h0))
    results = {}

    def on_done(c):
        assert c["status"] == sse.REQ_DONE
        results[c["id"]] = fetch(ctx, c)
        srv.release(c["id"])

    got = drain(srv, len(reqs), on_done)
    st = srv.stats()
    srv.stop()
    say(f"[serve] stats {st}")
    assert st["max_active_seen"] >= 3 and st["ticks"] >= 4
    for rid, r in zip(ids, ref):
        same(results[rid], r)
        assert got[rid]["histories"] == reqs[ids.index(rid)][1]
        assert got[rid]["t_submit"] <= got[rid]["t_admit"] <= got[rid]["t_complete"]
    same((own_c, own_w), ref[1])
    ctx.close()


def test_gap_model_requests_alone_and_in_the_mix():
    """With the gap model on (edge-LUT policy), the server's work-list
    kernels (the coincidence evaluation compiled with gaps) give every
    request the sinograms sse_simulate gives it alone."""
    import oracle as O
    ctx, pids = tiny_ctx()
    w = W.WORKLOADS["tiny"]
    dims = W.gap_lut_dims(w.scanner, w.lut_dims)
    ld, lut = W.make_lut(dims, 5)
    ctx.load_lut(ld, lut)
    gt, ga = W.edge_geometries(w.scanner, W.TINY_GAPS)
    ctx.set_gaps(W.gap_desc(W.TINY_GAPS, "edge_lut"), O.edge_lut(gt), O.edge_lut(ga))
    reqs = [(pids[0], 3_000_000, 21, 0), (pids[1], 170_000, 22, 0), (pids[0], 60_000, 23, 5_000)]
    ref = [alone(ctx, *r) for r in reqs]
    assert int(ref[0][0].sum()) > 0
    srv = sse.Server(ctx, max_active=4, tick_histories=1_000_000, chunk_histories=4096)
    ids = [srv.submit(pid, n, seed, h_offset=h0) for pid, n, seed, h0 in reqs]
    results = {}

    def on_done(c):
        assert c["status"] == sse.REQ_DONE
        results[c["id"]] = fetch(ctx, c)
        srv.release(c["id"])

    drain(srv, len(reqs), on_done)
    srv.stop()
    for rid, r in zip(ids, ref):
        same(results[rid], r)
    ctx.close()


def test_pair_pruning_requests_match_full_tracking():
    """With pair pruning on, the server's requests get the sinograms that
    sse_simulate gives them alone with both photons of every history
    tracked."""
    ctx, pids = tiny_ctx()
    reqs = [(pids[0], 3_000_000, 31, 0), (pids[1], 170_000, 32, 0), (pids[2], 90_000, 33, 0)]
    ref = [alone(ctx, *r) for r in reqs]
    ctx.set_pair_pruning(True)
    srv = sse.Server(ctx, max_active=4, tick_histories=1_000_000, chunk_histories=4096)
    ids = [srv.submit(pid, n, seed, h_offset=h0) for pid, n, seed, h0 in reqs]
    results = {}

    def on_done(c):
        assert c["status"] == sse.REQ_DONE
        results[c["id"]] = fetch(ctx, c)
        srv.release(c["id"])

    drain(srv, len(reqs), on_done)
    srv.stop()
    for rid, r in zip(ids, ref):
        same(results[rid], r)
    assert int(ref[0][0].sum()) > 0
    ctx.close()


def test_context_tables_are_locked_while_serving():
    """Calls that would replace or free device tables a running server's
    requests read are refused with SSE_EBUSY until the server stops."""
    ctx, pids = tiny_ctx()
    w = W.WORKLOADS["tiny"]
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    srv = sse.Server(ctx, max_active=2)
    try:
        for call in (lambda: ctx.load_lut(ld, lut), lambda: ctx.set_gaps(None),
                     lambda: ctx.update_activity(pids[0], W.tiny_cylinder()[2]),
                     lambda: ctx.unload_phantom(pids[2]), lambda: ctx.set_pair_pruning(True)):
            with pytest.raises(sse.SseError) as e:
                call()
            assert e.value.status == sse.EBUSY
        assert sse.lib().sse_destroy(ctx._h) == sse.EBUSY
    finally:
        srv.stop()
    ctx.load_lut(ld, lut)
    ctx.unload_phantom(pids[2])
    ctx.close()


def test_admission_by_hbm_budget():
    ctx, pids = tiny_ctx()
    footprint = ctx.n_bins * 12
    srv = sse.Server(ctx, max_active=8, hbm_budget_bytes=footprint, tick_histories=50_000, chunk_histories=4096)
    ids = [srv.submit(pids[i % 3], 60_000 + 1000 * i, 100 + i) for i in range(4)]
    results = {}

    def on_done(c):
        results[c["id"]] = fetch(ctx, c)
        srv.release(c["id"])   # frees the one buffer the budget allows

    drain(srv, 4, on_done)
    st = srv.stats()
    srv.stop()
    say(f"[serve] budget stats {st}")
    assert st["max_active_seen"] == 1
    assert st["bytes_allocated"] == footprint
    for i, rid in enumerate(ids):
        same(results[rid], alone(ctx, pids[i % 3], 60_000 + 1000 * i, 100 + i))
    with pytest.raises(sse.SseError) as e:
        s2 = sse.Server(ctx, max_active=2, hbm_budget_bytes=footprint // 2)
        try:
            s2.submit(pids[0], 10, 1)
        finally:
            s2.stop()
    assert e.value.status == sse.EBUSY
    ctx.close()


def test_phantom_loaded_while_serving_counts_against_the_budget():
    """A phantom loaded after the server started (the scheduler thread looks
    phantoms up meanwhile) is served, and its device memory counts against
    the HBM budget: a request whose outputs the budget held before no longer
    fits, while one with caller-owned outputs runs."""
    ctx, pids = tiny_ctx()
    footprint = ctx.n_bins * 12
    srv = sse.Server(ctx, max_active=2, hbm_budget_bytes=footprint + footprint // 2, tick_histories=50_000,
                     chunk_histories=4096)
    try:
        # 64 x 64 x 48 voxels of 2 mm: 13 bytes per voxel on the device (map,
        # alias column, palette index), about 1.4 footprints
        pd, mu, act = W.uniform_box(n=(64, 64, 48), voxel_mm=(2.0, 2.0, 2.0))
        pid = ctx.load_phantom(pd, mu, act)
        assert 64 * 64 * 48 * 13 > footprint // 2
        with pytest.raises(sse.SseError) as e:
            srv.submit(pid, 20_000, 7)
        assert e.value.status == sse.EBUSY
        out = ctx.new_outputs(stats=False)
        rid = srv.submit(pid, 20_000, 7, counts=out["scatter_counts"], weights=out["scatter_weights"])
        got = drain(srv, 1, lambda c: None)
        assert got[rid]["status"] == sse.REQ_DONE
        torch.cuda.synchronize()
        served = (out["scatter_counts"].clone(), out["scatter_weights"].clone())
    finally:
        srv.stop()
    same(served, alone(ctx, pid, 20_000, 7))
    ctx.close()


def test_cancel_and_errors():
    ctx, pids = tiny_ctx()
    srv = sse.Server(ctx, max_active=2, tick_histories=100_000, chunk_histories=8192)
    big = srv.submit(pids[0], 200_000_000, 5)
    small = srv.submit(pids[1], 50_000, 6)
    time.sleep(0.05)
    srv.cancel(big)
    got = {}

    def on_done(c):
        got[c["id"]] = c
        srv.release(c["id"])

    drain(srv, 2, on_done)
    assert got[big]["status"] == sse.REQ_CANCELLED and got[big]["histories"] < 200_000_000
    assert got[small]["status"] == sse.REQ_DONE and got[small]["histories"] == 50_000
    with pytest.raises(sse.SseError):
        srv.cancel(big)
    with pytest.raises(sse.SseError):
        srv.submit(999, 10, 1)
    with pytest.raises(sse.SseError):
        srv.submit(pids[0], 0, 1)
    with pytest.raises(sse.SseError):
        srv.submit(pids[0], 10, 1, counts=torch.zeros(ctx.n_bins, dtype=torch.int32, device="cuda"))
    # stop drains queued work
    for i in range(3):
        srv.submit(pids[i], 20_000, 40 + i)
    srv.stop()
    ctx.close()


def test_clinical_serving_phantoms_alone_and_in_the_mix():
    """Body-like serving phantoms of the three grid kinds on the Signa
    scanner and sinogram, mixed with different budgets."""
    w = W.WORKLOADS["clinical"]
    ctx = sse.Context(w.scanner, w.sino, w.physics)
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    ctx.load_lut(ld, lut)
    reqs = []
    for seed, n in ((1, 3_000_000), (2, 1_000_000), (5, 2_000_000)):
        pd, mu, act = W.serving_phantom(seed)
        reqs.append((ctx.load_phantom(pd, mu, act), n, 1000 + seed))
    srv = sse.Server(ctx, max_active=3, tick_histories=1_500_000)
    ids = [srv.submit(*r) for r in reqs]
    results = {}

    def on_done(c):
        results[c["id"]] = fetch(ctx, c)
        srv.release(c["id"])

    drain(srv, 3, on_done, timeout_s=300.0)
    srv.stop()
    for rid, r in zip(ids, reqs):
        same(results[rid], alone(ctx, *r))
    ctx.close()
