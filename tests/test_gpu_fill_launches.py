"""Fill launches of the production simulate: a run whose in-window pairs do
not fit the pair buffer goes through launches that each stop taking
histories when the buffer is nearly full, the next one going on from the
common claim cursor.  Every history draws from its own random stream, so the
sinograms cannot depend on how the run is cut into launches (Methods,
"Scatter simulator description": the simulated events are independent):
counts equal bit for bit, weights up to the order of their binary64 sums."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from tests import harness as H  # noqa: E402


def run(ctx, pid, n, seed, max_records=None):
    if max_records is not None:
        ctx.set_pair_buffer(max_records)
    out = ctx.new_outputs(trues=True)
    ctx.simulate(pid, n, seed, out)
    torch.cuda.synchronize()
    got = {k: v.cpu().numpy() for k, v in out.items()}
    del out
    return got


def test_fill_launches_resume_where_the_buffer_filled():
    case = H.case_from("clinical")
    ctx, pid = H.open_context(case)
    n, seed = 1_200_000_000, 4242
    small = 14 << 20  # fill launches: above the fill threshold of an MI355X (13.8 M records)
    try:
        print(f"[fill] clinical, {n} histories, default buffer", flush=True)
        a = run(ctx, pid, n, seed)
        print(f"[fill] pair buffer of {small} records", flush=True)
        b = run(ctx, pid, n, seed, small)
        print("[fill] pair buffer of 4 Mi records (launches sized for the worst case)", flush=True)
        c = run(ctx, pid, n, seed, 4 << 20)
    finally:
        ctx.close()
    # every counted pair went through the buffer, so a buffer of `small`
    # records could not have carried the run in one launch
    counted = int(a["scatter_counts"].sum(dtype=np.int64) + a["true_counts"].sum(dtype=np.int64))
    assert counted > small, counted
    for o in (b, c):
        assert np.array_equal(o["scatter_counts"], a["scatter_counts"])
        assert np.array_equal(o["true_counts"], a["true_counts"])
        np.testing.assert_allclose(o["scatter_weights"], a["scatter_weights"], rtol=1e-12, atol=0)
        np.testing.assert_allclose(o["true_weights"], a["true_weights"], rtol=1e-12, atol=0)
