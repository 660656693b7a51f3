"""The allocation-free simulate (sse_simulate_noalloc) against sse_simulate:
two calls in a row through the C ABI, the second with a smaller input, each
giving the sinograms sse_simulate gives for the same histories (counts bit
for bit, weights within 1e-12 relative: only the order of the binary64 sums
differs).  The clinical call is longer than one launch's share of the
static scratch, so it also covers the split into several launches."""
import sys

import numpy as np
import pytest

import workloads as W
from tests import harness as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2509_05047_amd as sse  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _same(a, b, names):
    for cn, wn in names:
        assert torch.equal(a[cn], b[cn]), cn
        nz = b[wn] != 0
        assert torch.equal(a[wn] != 0, nz), wn
        if nz.any():
            rel = float(((a[wn][nz] - b[wn][nz]).abs() / b[wn][nz].abs()).max())
            assert rel <= 1e-12, (wn, rel)


def _run(ctx, pid, n, seed, h0, trues, noalloc):
    out = ctx.new_outputs(trues=trues, stats=False)
    if noalloc:
        ctx.simulate_noalloc(pid, n, seed, out, h_offset=h0)
    else:
        ctx.simulate(pid, n, seed, out, h_offset=h0)
    torch.cuda.synchronize()
    return out


def test_noalloc_equals_simulate_on_two_calls_in_a_row():
    case = H.case_from("clinical")
    ctx, pid = H.open_context(case)
    try:
        # clinical body, 6e6 histories with trues, then 150 001 histories
        # without trues at another offset (the scratch keeps the first
        # call's contents)
        calls = [(6_000_000, 5678, 1_000_000, True), (150_001, 91, 12_345_678, False)]
        for n, seed, h0, trues in calls:
            say(f"[noalloc] clinical n={n} seed={seed} h0={h0} trues={trues}")
            a = _run(ctx, pid, n, seed, h0, trues, noalloc=True)
            b = _run(ctx, pid, n, seed, h0, trues, noalloc=False)
            names = [("scatter_counts", "scatter_weights")]
            if trues:
                names.append(("true_counts", "true_weights"))
            _same(a, b, names)
            say(f"[noalloc] {int(b['scatter_counts'].sum())} scatter coincidences, identical")
            del a, b
    finally:
        ctx.close()


def test_noalloc_refuses_statistics_and_records():
    case = H.case_from("tiny")
    ctx, pid = H.open_context(case)
    try:
        out = ctx.new_outputs(stats=True)
        with pytest.raises(sse.SseError) as e:
            ctx.simulate_noalloc(pid, 1000, 1, out)
        assert e.value.status == sse.EINVAL
        out = ctx.new_outputs(records=10)
        with pytest.raises(sse.SseError) as e:
            ctx.simulate_noalloc(pid, 10, 1, out)
        assert e.value.status == sse.EINVAL
        # zero histories: nothing to do
        out = ctx.new_outputs()
        ctx.simulate_noalloc(pid, 0, 1, out)
        torch.cuda.synchronize()
        assert int(out["scatter_counts"].sum()) == 0
    finally:
        ctx.close()


def test_noalloc_tiny_workload_equals_simulate_and_repeats():
    """The whole tiny workload twice in a row through the allocation-free
    call: both equal sse_simulate, so nothing of the first call leaks into
    the second through the shared scratch."""
    case = H.case_from("tiny")
    ctx, pid = H.open_context(case)
    try:
        w = W.WORKLOADS["tiny"]
        b = _run(ctx, pid, w.n_histories, w.seed, 0, True, noalloc=False)
        for _ in range(2):
            a = _run(ctx, pid, w.n_histories, w.seed, 0, True, noalloc=True)
            _same(a, b, [("scatter_counts", "scatter_weights"), ("true_counts", "true_weights")])
        say(f"[noalloc] tiny: {int(b['scatter_counts'].sum())} scatter, {int(b['true_counts'].sum())} true")
        assert np.isfinite(float(b["true_weights"].sum()))
    finally:
        ctx.close()
