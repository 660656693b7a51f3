"""Parity of the HIP path (through the C ABI) with the CPU oracle.

Bar: at least 99.9 % of histories identical (all 32 record words, bit for
bit), integer count sinograms bit-exact over the identical histories, and
binary64 weight sinograms within 1e-5 relative per bin (the only expected
difference is the order of the binary64 sums, relative error below
n_bin * 2^-53).
"""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import post
import workloads as W
from tests import harness as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2509_05047_amd as sse  # noqa: E402


def stats_match(g, o):
    """Every statistic equal, the Philox block count included: the kernel
    counts the blocks a history uses (its words consumed, rounded up to
    whole blocks), which is what the oracle's on-demand generator makes."""
    assert dict(g) == dict(o), {k: (g[k], o[k]) for k in g if g[k] != o.get(k)}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def check_case(case, n, seed, h_offset=0, stride=1, min_identical=0.999):
    say(f"[parity] n={n} seed={seed} h0={h_offset} stride={stride} lut_dtype={case.lut_dtype}")
    ctx, pid = H.open_context(case)
    try:
        g = H.run_gpu(ctx, pid, n, seed, h_offset=h_offset, record_stride=stride)
    finally:
        ctx.close()
    if stride == 1:
        o = H.run_oracle(case, n, seed, h_offset=h_offset)
    else:
        hs = np.arange(h_offset, h_offset + n, stride, dtype=np.uint64)
        o = H.run_oracle(case, 0, seed, h_list=hs, sinograms=False, trues=False)
    same = H.identical_mask(g["records"], o["records"])
    frac = same.mean()
    say(f"[parity] identical histories {frac:.6f} ({(~same).sum()} differ); gpu {g['seconds']:.3f}s")
    assert frac >= min_identical, H.describe_mismatch(g["records"], o["records"])
    return g, o, same


def test_tiny_workload_full_parity():
    case = H.case_from("tiny")
    w = W.WORKLOADS["tiny"]
    g, o, same = check_case(case, w.n_histories, w.seed)
    worst = H.compare_sinograms(g, o, g["records"], o["records"], same)
    say(f"[parity] worst relative weight difference {worst:.3e}")
    if same.all():
        stats_match(g["stats"], o["stats"])
    assert g["scatter_counts"].sum() > 0


@pytest.mark.parametrize("mode", ["lut5d_paper", "lut3d_angles", "lut3d_crystals", "lut1d", "nolut"])
def test_lut_modes_full_parity(mode):
    """The paper's LUT variants (unit dimensions of the 5D index) with its
    LUT energy configuration (0.1 % blur, 300-650 keV), and the no-LUT mode
    (11.2 % blur, 425-650 keV, weight 1), on the whole tiny workload."""
    w = W.WORKLOADS["tiny"]
    phys, ld, lut = W.lut_mode(w, mode)
    case = H.case_from("tiny", physics=phys, lut=(ld, lut))
    g, o, same = check_case(case, w.n_histories, w.seed)
    assert same.all()
    worst = H.compare_sinograms(g, o, g["records"], o["records"], same)
    say(f"[parity] {mode}: worst relative weight difference {worst:.3e}")
    stats_match(g["stats"], o["stats"])
    assert g["scatter_counts"].sum() > 0
    if mode == "nolut":
        assert np.array_equal(g["scatter_weights"], g["scatter_counts"].astype(np.float64))


@pytest.mark.parametrize("policy", ["discard", "nearest", "edge_lut"])
def test_gap_policies_full_parity(policy):
    """Gaps between modules and blocks with each gap policy (the LUT with
    its virtual gap indices; the oracle's edge LUTs), TOF jitter on so that
    the jitter continues the stream after the edge draws: the whole tiny
    workload history by history."""
    w = W.WORKLOADS["tiny"]
    case = H.with_gaps(H.case_from("tiny", tof_sigma=15.0), W.TINY_GAPS, policy)
    g, o, same = check_case(case, w.n_histories, w.seed)
    assert same.all()
    worst = H.compare_sinograms(g, o, g["records"], o["records"], same)
    say(f"[parity] gaps {policy}: worst relative weight difference {worst:.3e}, "
        f"rej_gap {g['stats']['rej_gap']}, gap_assigned {g['stats']['gap_assigned']}")
    stats_match(g["stats"], o["stats"])
    assert (g["stats"]["rej_gap"] > 0) == (policy == "discard")
    assert (g["stats"]["gap_assigned"] > 0) == (policy != "discard")


def test_gap_edge_lut_clinical_slice_parity():
    """The Signa-like scanner with its gaps, the paper's LUT shape on the
    crystal axes (18 transaxial, 55 axial indices) and the edge-crystal LUT
    policy, with the edge LUTs the library builds itself."""
    import paper_2509_05047_amd as lib_sse
    base = H.case_from("clinical")
    gt, ga = W.edge_geometries(base.scanner, W.SIGNA_GAPS)
    orc_edge = (O.edge_lut(gt), O.edge_lut(ga))
    # the two builders agree to float rounding; both sides then use the oracle's tables
    assert max(np.abs(lib_sse.build_edge_lut(gt) - orc_edge[0]).max(),
               np.abs(lib_sse.build_edge_lut(ga) - orc_edge[1]).max()) < 2e-7
    case = H.with_gaps(base, W.SIGNA_GAPS, "edge_lut", edge=orc_edge)
    assert case.lut_desc.dims[3:] == (18, 55)
    g, o, same = check_case(case, 200_003, 5678, h_offset=987_654_321)
    H.compare_sinograms(g, o, g["records"], o["records"], same)
    if same.all():
        stats_match(g["stats"], o["stats"])
    say(f"[parity] clinical gaps: {same.mean():.6f} identical, gap_assigned {g['stats']['gap_assigned']}")


def test_paper_size_lut_with_gaps():
    """The LUT at the paper's shape on the Signa-like scanner with gaps: 5 keV
    energy bins over 300-650 keV, 5 degree angle bins, 18 transaxial and 55
    axial crystal indices (70 x 36 x 36 x 18 x 55 = 90 M entries, FP16), the
    paper's LUT energy setting and the edge-LUT policy."""
    w = W.WORKLOADS["clinical"]
    dims = (70, 36, 36, 18, 55)
    assert dims == W.gap_lut_dims(w.scanner, (70, 36, 36, 16, 45))
    ld, vals = W.make_lut(dims, 11, e_min=300.0, e_max=650.0)
    store = vals.astype(np.float16).view(np.uint16)
    seen = vals.astype(np.float16).astype(np.float32)
    base = H.case_from("clinical", physics=dict(W.PHYSICS_LUT_PAPER))
    case = H.with_gaps(base, W.SIGNA_GAPS, "edge_lut")
    case.lut_desc, case.lut, case.lut_store, case.lut_dtype = ld, seen, store, sse.F16
    g, o, same = check_case(case, 100_003, 31, h_offset=4_000_000_000)
    H.compare_sinograms(g, o, g["records"], o["records"], same)
    if same.all():
        stats_match(g["stats"], o["stats"])
    lidx = g["records"]["ph"]["lut_index"]
    used = lidx[lidx != 0xFFFFFFFF]
    say(f"[parity] paper-size LUT: max index {int(used.max())} of {vals.size}")
    assert int(used.max()) > vals.size // 2


def test_clinical_slice_parity_with_offset_and_ragged_count():
    case = H.case_from("clinical")
    g, o, same = check_case(case, 200_003, 5678, h_offset=123_456_789)
    H.compare_sinograms(g, o, g["records"], o["records"], same)
    if same.all():
        stats_match(g["stats"], o["stats"])


def test_clinical_no_jitter_parity():
    case = H.case_from("clinical", tof_sigma=0.0)
    g, o, same = check_case(case, 50_000, 99)
    H.compare_sinograms(g, o, g["records"], o["records"], same)


@pytest.mark.parametrize("dtype", [sse.F16, sse.BF16])
def test_narrow_lut_parity(dtype):
    """FP16 / BF16 LUT: the oracle sees the dequantised values; histories and
    weights match exactly."""
    case = H.case_from("clinical", lut_dtype=dtype)
    g, o, same = check_case(case, 50_000, 4242)
    H.compare_sinograms(g, o, g["records"], o["records"], same)


def test_full_size_clinical_sampled_histories():
    """The clinical workload at its full size (1e9 histories).  The
    instrumented launch records every 10 000th history, which the oracle
    recomputes one by one; the production launch the benchmark times (no
    statistics, no records) must then give the same sinograms."""
    case = H.case_from("clinical")
    w = W.WORKLOADS["clinical"]
    g, o, same = check_case(case, w.n_histories, w.seed, stride=10_000)
    st = g["stats"]
    assert st["histories"] == w.n_histories
    assert int(g["scatter_counts"].sum()) == st["scatter"]
    assert int(g["true_counts"].sum()) == st["true"]
    assert np.all(g["scatter_weights"] <= g["scatter_counts"] * (1 + 1e-12))
    say(f"[full] instrumented {w.n_histories / g['seconds']:.3e} histories/s, scatter {st['scatter']}, trues {st['true']}")
    ctx, pid = H.open_context(case)
    try:
        prod = H.run_gpu(ctx, pid, w.n_histories, w.seed, stats=False)
        # the benchmark's launch: scatter sinogram only
        bench_like = H.run_gpu(ctx, pid, w.n_histories, w.seed, stats=False, trues=False)
        ctx.set_pair_pruning(True)
        pruned = H.run_gpu(ctx, pid, w.n_histories, w.seed, stats=False)
    finally:
        ctx.close()
    say(f"[full] production {w.n_histories / prod['seconds']:.3e} histories/s, "
        f"scatter only {w.n_histories / bench_like['seconds']:.3e}, "
        f"with pair pruning {w.n_histories / pruned['seconds']:.3e}")
    for run in (prod, bench_like, pruned):
        for c, wt in (("scatter_counts", "scatter_weights"), ("true_counts", "true_weights")):
            if run.get(c) is None:
                continue
            assert np.array_equal(run[c], g[c]), c
            nz = g[wt] != 0
            assert np.array_equal(run[wt] != 0, nz)
            assert np.max(np.abs(run[wt][nz] - g[wt][nz]) / g[wt][nz]) < 1e-12


@pytest.mark.parametrize("policy", [None, "discard", "edge_lut"])
def test_pair_pruning_keeps_sinograms(policy):
    """Pair pruning (photon B not tracked once photon A ended outside the
    energy window), and production launches without a trues sinogram (which
    queue only scattered pairs): the sinograms equal the oracle's full
    simulation of every history (counts bit for bit, weights within the
    bar), with and without gaps and with TOF jitter, so that the coincidence
    draws continue the stream where photon B left it; the instrumented
    launch still tracks both photons."""
    w = W.WORKLOADS["tiny"]
    case = H.case_from("tiny", tof_sigma=15.0)
    if policy is not None:
        case = H.with_gaps(case, W.TINY_GAPS, policy)
    o = H.run_oracle(case, w.n_histories, w.seed)
    ctx, pid = H.open_context(case)
    try:
        full = H.run_gpu(ctx, pid, w.n_histories, w.seed, stats=False)
        # without a trues sinogram the production launch queues only the
        # scattered pairs
        scatter_only = H.run_gpu(ctx, pid, w.n_histories, w.seed, stats=False, trues=False)
        ctx.set_pair_pruning(True)
        pruned = H.run_gpu(ctx, pid, w.n_histories, w.seed, stats=False)
        pruned_scatter_only = H.run_gpu(ctx, pid, w.n_histories, w.seed, stats=False, trues=False)
        inst = H.run_gpu(ctx, pid, w.n_histories, w.seed, record_stride=1)
        ctx.set_pair_pruning(False)
        again = H.run_gpu(ctx, pid, w.n_histories, w.seed, stats=False)
    finally:
        ctx.close()
    same = H.identical_mask(inst["records"], o["records"])
    assert same.all(), H.describe_mismatch(inst["records"], o["records"])
    stats_match(inst["stats"], o["stats"])
    for run in (full, scatter_only, pruned, pruned_scatter_only, again):
        H.compare_sinograms(run, o, o["records"], o["records"], same)
    assert scatter_only.get("true_counts") is None
    assert np.array_equal(pruned["scatter_counts"], full["scatter_counts"])
    assert int(o["scatter_counts"].sum()) > 0 and int(o["true_counts"].sum()) > 0
    say(f"[pruning] gaps {policy}: {int(o['scatter_counts'].sum())} scatter, "
        f"{int(o['true_counts'].sum())} true coincidences, "
        f"{o['stats']['in_window'] / w.n_histories:.3f} singles in the window per history")


def test_pair_pruning_argument_checks():
    case = H.case_from("tiny")
    ctx, pid = H.open_context(case)
    try:
        lib = sse.lib()
        assert lib.sse_set_pair_pruning(ctx._h, 2) == 1  # SSE_EINVAL
        assert lib.sse_set_pair_pruning(None, 1) == 1
        assert lib.sse_set_pair_pruning(ctx._h, 1) == 0
        assert lib.sse_set_pair_pruning(ctx._h, 0) == 0
    finally:
        ctx.close()


def test_split_runs_sum_to_whole_run_and_repeat():
    case = H.case_from("tiny")
    ctx, pid = H.open_context(case)
    try:
        whole = H.run_gpu(ctx, pid, 60_000, 77)
        again = H.run_gpu(ctx, pid, 60_000, 77)
        out = ctx.new_outputs(trues=True)
        for h0, n in ((0, 12_345), (12_345, 40_000), (52_345, 7_655)):
            ctx.simulate(pid, n, 77, out, h_offset=h0)
        torch.cuda.synchronize()
    finally:
        pass
    parts_c = out["scatter_counts"].cpu().numpy().view(np.uint32)
    parts_w = out["scatter_weights"].cpu().numpy()
    assert np.array_equal(parts_c, whole["scatter_counts"])
    assert np.array_equal(again["scatter_counts"], whole["scatter_counts"])
    nz = whole["scatter_weights"] != 0
    assert np.max(np.abs(parts_w[nz] - whole["scatter_weights"][nz]) / whole["scatter_weights"][nz]) < 1e-12
    ctx.close()


def test_results_do_not_depend_on_statistics_output():
    """Sinograms and records are the same whether or not the statistics
    counters are requested."""
    case = H.case_from("clinical")
    ctx, pid = H.open_context(case)
    try:
        a = ctx.new_outputs(trues=True, stats=True, records=2000, record_stride=25)
        b = ctx.new_outputs(trues=True, stats=False, records=2000, record_stride=25)
        ctx.simulate(pid, 50_000, 31, a)
        ctx.simulate(pid, 50_000, 31, b)
        torch.cuda.synchronize()
        for k in ("scatter_counts", "true_counts", "records"):
            assert torch.equal(a[k], b[k]), k
        for k in ("scatter_weights", "true_weights"):
            assert torch.allclose(a[k], b[k], rtol=1e-12, atol=0), k
    finally:
        ctx.close()


@pytest.mark.parametrize("h_offset", [(1 << 32) - 40_000, (1 << 40) + 12_345, (1 << 63) - 100_003])
def test_history_indices_beyond_32_bits(h_offset):
    """History indices whose upper 32 bits are not zero (the second counter
    word of the stream), a range that crosses 2^32, and the top of the index
    range: every history identical to the oracle's."""
    case = H.case_from("tiny", tof_sigma=15.0)
    g, o, same = check_case(case, 100_003, 4242, h_offset=h_offset)
    assert same.all()
    H.compare_sinograms(g, o, g["records"], o["records"], same)
    stats_match(g["stats"], o["stats"])


def test_edge_cases():
    case = H.case_from("tiny")
    ctx, pid = H.open_context(case)
    try:
        # zero histories: nothing happens
        z = H.run_gpu(ctx, pid, 0, 1)
        assert z["scatter_counts"].sum() == 0 and z["stats"]["histories"] == 0
        # one history
        one = H.run_gpu(ctx, pid, 1, 1, h_offset=5, record_stride=1)
        o = H.run_oracle(case, 1, 1, h_offset=5)
        assert H.identical_mask(one["records"], o["records"]).all()
        # simulate before a phantom id exists
        with pytest.raises(sse.SseError) as e:
            ctx.simulate(999, 10, 1, ctx.new_outputs())
        assert e.value.status == sse.EINVAL
        # record stride 0 with records
        bad = ctx.new_outputs(records=4)
        bad["record_stride"] = 0
        with pytest.raises(sse.SseError):
            ctx.simulate(pid, 4, 1, bad)
    finally:
        ctx.close()
    # no LUT loaded
    ctx = sse.Context(case.scanner, case.sino, case.physics)
    try:
        pid = ctx.load_phantom(case.pdesc, case.mu, case.act)
        with pytest.raises(sse.SseError) as e:
            ctx.simulate(pid, 10, 1, ctx.new_outputs())
        assert e.value.status == sse.ESTATE
        # invalid phantom inputs
        with pytest.raises(sse.SseError):
            ctx.load_phantom(case.pdesc, -case.mu, case.act)
        with pytest.raises(sse.SseError):
            ctx.load_phantom(case.pdesc, case.mu, np.zeros_like(case.act))
        big = W.centred_desc((200, 200, 4), (4.0, 4.0, 4.0))
        with pytest.raises(sse.SseError):
            ctx.load_phantom(big, np.zeros(big.shape, np.float32), np.ones(big.shape, np.float32))
        with pytest.raises(sse.SseError):
            ctx.load_lut(case.lut_desc, case.lut * 2.0)
    finally:
        ctx.close()


def test_gap_argument_checks():
    """sse_set_gaps and the LUT-layout checks reject what the gap model
    cannot take, and switching gaps off restores the plain cylinder."""
    case = H.case_from("tiny")
    gcase = H.with_gaps(case, W.TINY_GAPS, "edge_lut")
    tab = gcase.edge_t
    ctx, pid = H.open_context(case)
    try:
        bad = [dict(W.TINY_GAPS, policy=3), dict(W.TINY_GAPS, policy="nearest", transaxial_gap_rad=1.0),
               dict(W.TINY_GAPS, policy="nearest", axial_gap_mm=-1.0),
               dict(W.TINY_GAPS, policy="nearest", axial_gap_mm=500.0)]
        for g in bad:
            with pytest.raises(sse.SseError) as e:
                ctx.set_gaps(g)
            assert e.value.status == sse.EINVAL
        # the plain LUT (4 x 2 crystal axes) lacks the gap layout
        with pytest.raises(sse.SseError) as e:
            ctx.set_gaps(W.gap_desc(W.TINY_GAPS, "nearest"))
        assert e.value.status == sse.EINVAL
        # load the gap-layout LUT, then the edge policy needs both tables in [0, 1]
        ctx.load_lut(gcase.lut_desc, gcase.lut_store)
        with pytest.raises(sse.SseError):
            ctx.set_gaps(gcase.gaps, tab, None)
        with pytest.raises(sse.SseError):
            ctx.set_gaps(gcase.gaps, tab, tab * 2.0)
        ctx.set_gaps(gcase.gaps, gcase.edge_t, gcase.edge_a)
        # with gaps on, a LUT without the layout is refused
        with pytest.raises(sse.SseError):
            ctx.load_lut(case.lut_desc, case.lut_store)
        g = H.run_gpu(ctx, pid, 20_000, 5, record_stride=1)
        o = H.run_oracle(gcase, 20_000, 5)
        assert H.identical_mask(g["records"], o["records"]).all()
        # gaps off again, the original LUT: the plain run
        ctx.set_gaps(None)
        ctx.load_lut(case.lut_desc, case.lut_store)
        g = H.run_gpu(ctx, pid, 20_000, 5, record_stride=1)
        o = H.run_oracle(case, 20_000, 5)
        assert H.identical_mask(g["records"], o["records"]).all()
    finally:
        ctx.close()


def test_large_grid_index_paths():
    """A 1 x 4100 x 4100 grid: ny nz > 2^24 takes the 32-bit voxel index
    (not the 24-bit multiplies) and nvox >= 2^24 the integer-division voxel
    decomposition of the emission; histories match the oracle."""
    desc = W.centred_desc((1, 4100, 4100), (100.0, 0.05, 0.05))
    z, y, x = W.voxel_centres(desc)
    mu = np.broadcast_to(np.where((y * y + z * z) <= 60.0 ** 2, W.MU_WATER, 0.0), desc.shape).astype(np.float32)
    act = np.broadcast_to(np.where((y * y + z * z) <= 50.0 ** 2, 1.0, 0.0), desc.shape).astype(np.float32)
    case = H.case_from("tiny", phantom=(desc, mu, act))
    assert desc.ny * desc.nz > (1 << 24)
    g, o, same = check_case(case, 20_000, 17)
    assert same.all()
    H.compare_sinograms(g, o, g["records"], o["records"], same)


def test_device_division_is_correctly_rounded():
    """The transport's device division (refined reciprocal, one remainder
    correction) equals the IEEE quotient: its reciprocal is the correctly
    rounded 1/b for every significand, and 2^31 hashed quotients match."""
    case = H.case_from("tiny")
    ctx = sse.Context(case.scanner, case.sino, case.physics)
    try:
        for seed in (1, 2):
            r, q = ctx.check_division(1 << 30, seed)
            say(f"[division] seed {seed}: reciprocal mismatches {r} of 2^23, quotient mismatches {q} of 2^30")
            assert r == 0 and q == 0
    finally:
        ctx.close()


def test_point_source_and_all_ones_lut():
    w = W.WORKLOADS["tiny"]
    ones_case = H.case_from("tiny")
    ones_case.lut = np.ones(ones_case.lut_desc.dims, np.float32)
    ones_case.lut_store = ones_case.lut
    ctx, pid = H.open_context(ones_case)
    try:
        g = H.run_gpu(ctx, pid, 100_000, 3)
    finally:
        ctx.close()
    assert np.array_equal(g["scatter_weights"], g["scatter_counts"].astype(np.float64))
    assert np.array_equal(g["true_weights"], g["true_counts"].astype(np.float64))
    src = H.case_from("tiny", phantom=W.point_source((0.0, 0.0, 0.0)))
    ctx, pid = H.open_context(src)
    try:
        g = H.run_gpu(ctx, pid, 50_000, 3, record_stride=1)
    finally:
        ctx.close()
    o = H.run_oracle(src, 50_000, 3)
    assert H.identical_mask(g["records"], o["records"]).all()
    assert g["scatter_counts"].sum() == 0 and g["true_counts"].sum() > 10_000
    assert w.scanner.n_crystals == 64


@pytest.mark.parametrize("sens_tof", [True, False])
def test_apply_sensitivity_bit_exact(sens_tof):
    case = H.case_from("tiny")
    rng = np.random.default_rng(1)
    sino = case.sino
    W_ = rng.uniform(0, 50, sino.n_bins)
    sens = W.make_sensitivity(sino, seed=3, tof_axis=sens_tof)
    ctx, pid = H.open_context(case, sensitivity=sens, sens_tof=sens_tof)
    try:
        dW = torch.from_numpy(W_).cuda()
        out = torch.empty(sino.n_bins, dtype=torch.float32, device="cuda")
        ctx.apply_sensitivity(dW, 0.37, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
    finally:
        ctx.close()
    ref = post.apply_sensitivity(W_.reshape(sino.shape), 0.37, sens).ravel()
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("which", ["tiny", "clinical"])
@pytest.mark.parametrize("sens_tof", [True, False])
def test_total_scatter_matches_oracle(which, sens_tof):
    """The device's binary64 total of scale * W * sens against the exact sum
    of the same products (tiny) or numpy's pairwise sum (clinical shape):
    relative 1e-12, and the same bits on a second call."""
    case = H.case_from(which)
    sino = case.sino
    rng = np.random.default_rng(5)
    W_ = rng.uniform(0, 50, sino.n_bins)
    W_[rng.random(sino.n_bins) < 0.5] = 0.0
    sens = W.make_sensitivity(sino, seed=3, tof_axis=sens_tof)
    ctx, pid = H.open_context(case, sensitivity=sens, sens_tof=sens_tof)
    try:
        dW = torch.from_numpy(W_).cuda()
        a = ctx.total_scatter(dW, 0.37)
        b = ctx.total_scatter(dW, 0.37)
        torch.cuda.synchronize()
        got, again = float(a.item()), float(b.item())
    finally:
        ctx.close()
    if which == "tiny":
        ref = post.total_scatter(W_.reshape(sino.shape), 0.37, sens)
    else:
        s = sens.astype(np.float64)
        ref = float(((0.37 * W_.reshape(sino.shape)) * (s if sens_tof else s[None])).sum())
    assert got == again
    assert abs(got - ref) <= 1e-12 * abs(ref), (got, ref)


@pytest.mark.parametrize("sigma", [(2.0, 2.0, 2.0), (3.8, 2.5, 4.5), (0.0, 1.5, 0.0), (1.0, 0.0, 0.0)])
def test_smoothing_matches_oracle(sigma):
    case = H.case_from("tiny")
    sino = case.sino
    x = np.random.default_rng(2).uniform(0, 1, sino.shape).astype(np.float32)
    ref = post.gaussian_smooth(x, sigma)
    ctx, pid = H.open_context(case)
    try:
        dx = torch.from_numpy(x.ravel()).cuda()
        out = torch.empty_like(dx)
        ctx.gaussian_smooth(dx, out, sigma)
        ctx.gaussian_smooth(dx, dx, sigma)  # in place
        torch.cuda.synchronize()
        got, inplace = out.cpu().numpy(), dx.cpu().numpy()
    finally:
        ctx.close()
    assert np.array_equal(got, inplace)
    rel = np.abs(got - ref.ravel()) / np.abs(ref.ravel())
    assert rel.max() < 1e-5, rel.max()


def test_clinical_finalize_matches_oracle_on_sampled_bins():
    """Full clinical sinogram shape: sensitivity times smoothed scaled
    weights (sigma 2 bins), checked on 2000 sampled bins."""
    case = H.case_from("clinical")
    sino = case.sino
    rng = np.random.default_rng(4)
    Wd = torch.rand(sino.n_bins, dtype=torch.float64, device="cuda") * 10.0
    sens = W.make_sensitivity(sino, seed=3, tof_axis=False)
    ctx, pid = H.open_context(case, sensitivity=sens, sens_tof=False)
    try:
        out = torch.empty(sino.n_bins, dtype=torch.float32, device="cuda")
        ctx.finalize(Wd, 0.5, out, sigma_bins=(2.0, 2.0, 2.0))
        torch.cuda.synchronize()
        scaled = (0.5 * Wd).float().cpu().numpy().reshape(sino.shape)
        got = out.cpu().numpy().reshape(sino.shape)
    finally:
        ctx.close()
    pts = np.stack([rng.integers(0, s, 2000) for s in sino.shape], 1)
    pts[:50, 2] = 0          # seam
    pts[50:100, 3] = 0       # radial edge
    pts[100:150, 1] = sino.n_plane - 1
    ref = post.gaussian_smooth_at(scaled, (2.0, 2.0, 2.0), pts) * sens[pts[:, 1], pts[:, 2], pts[:, 3]]
    g = got[pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]]
    assert np.max(np.abs(g - ref) / np.abs(ref)) < 1e-5


PAPER_SIGMA = tuple(f / 2.35482 for f in (9.0, 6.0, 10.5))   # FWHM [9, 6, 10.5] rad/view/plane bins


def _pattern(shape, seed):
    """Seeded multiplicative detector-like pattern (per radial bin and view)."""
    rng = np.random.default_rng(seed)
    nt, npl, nv, nr = shape
    p = (1.0 + 0.3 * rng.uniform(-1, 1, nr))[None, None, None, :] * (1.0 + 0.2 * rng.uniform(-1, 1, nv))[None, None, :, None]
    return np.broadcast_to(p, shape).astype(np.float64)


def test_smoothing_normalisation_workflow_matches_oracle_tiny():
    """The smoothing normalisation of a structured reference sinogram (heavy
    smoothing), then the normalised finalize of another sinogram with the
    paper's FWHM, on the whole tiny sinogram."""
    case = H.case_from("tiny")
    sino = case.sino
    rng = np.random.default_rng(8)
    P = _pattern(sino.shape, 9)
    Wref = P * rng.uniform(0.5, 1.5, sino.shape)
    Wref[0, 0, 0, :4] = 0.0
    Wobj = P * rng.uniform(0.0, 2.0, sino.shape)
    sens = W.make_sensitivity(sino, seed=3, tof_axis=False)
    heavy = tuple(3 * s for s in PAPER_SIGMA)
    ctx, pid = H.open_context(case, sensitivity=sens, sens_tof=False)
    try:
        dref = torch.from_numpy(Wref.ravel()).cuda()
        dobj = torch.from_numpy(Wobj.ravel()).cuda()
        norm = torch.empty(sino.n_bins, dtype=torch.float32, device="cuda")
        out = torch.empty(sino.n_bins, dtype=torch.float32, device="cuda")
        ctx.smoothing_normalisation(dref, 0.25, norm, heavy)
        torch.cuda.synchronize()
        got_n = norm.cpu().numpy().reshape(sino.shape)
        # the finalize gets the oracle's normalisation (rounded to binary32)
        # as its input on both sides
        ref_n = post.smoothing_normalisation(Wref, 0.25, heavy)
        n32 = ref_n.astype(np.float32)
        dn = torch.from_numpy(n32.ravel()).cuda()
        ctx.finalize_normalised(dobj, 0.5, dn, out, PAPER_SIGMA)
        torch.cuda.synchronize()
        got = out.cpu().numpy().reshape(sino.shape)
    finally:
        ctx.close()
    empty = Wref == 0
    assert np.all(got_n[empty] == 1.0)
    assert np.max(np.abs(got_n - ref_n) / ref_n) < 1e-5
    ref = post.finalize_normalised(Wobj, 0.5, n32.astype(np.float64), PAPER_SIGMA, sens)
    assert np.max(np.abs(got - ref) / np.abs(ref)) < 1e-5


def test_clinical_normalised_finalize_matches_oracle_on_sampled_bins():
    """Full clinical sinogram shape, paper FWHM, a seeded normalisation:
    sens * G(S * N) / N checked on 2000 sampled bins (seam and edges
    included)."""
    case = H.case_from("clinical")
    sino = case.sino
    rng = np.random.default_rng(5)
    Wd = torch.rand(sino.n_bins, dtype=torch.float64, device="cuda") * 10.0
    N = (1.0 / _pattern(sino.shape, 6)).astype(np.float32)
    sens = W.make_sensitivity(sino, seed=3, tof_axis=False)
    ctx, pid = H.open_context(case, sensitivity=sens, sens_tof=False)
    try:
        dn = torch.from_numpy(N.ravel()).cuda()
        out = torch.empty(sino.n_bins, dtype=torch.float32, device="cuda")
        ctx.finalize_normalised(Wd, 0.5, dn, out, PAPER_SIGMA)
        torch.cuda.synchronize()
        scaled = (0.5 * Wd).float().cpu().numpy().reshape(sino.shape).astype(np.float64)
        got = out.cpu().numpy().reshape(sino.shape)
    finally:
        ctx.close()
    pts = np.stack([rng.integers(0, s, 2000) for s in sino.shape], 1)
    pts[:50, 2] = 0
    pts[50:100, 3] = 0
    pts[100:150, 1] = sino.n_plane - 1
    x = scaled * N.astype(np.float64)
    ref = (post.gaussian_smooth_at(x, PAPER_SIGMA, pts) / N[pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]]
           * sens[pts[:, 1], pts[:, 2], pts[:, 3]])
    g = got[pts[:, 0], pts[:, 1], pts[:, 2], pts[:, 3]]
    assert np.max(np.abs(g - ref) / np.abs(ref)) < 1e-5


def test_precision_forms_against_fp64_oracle():
    """Narrow-LUT precision forms (config C3) against the FP64 oracle with the
    FP32 LUT.  Bounds: with the same dequantised LUT the binary32 path equals
    the binary32 oracle up to binary64 summation order (<= 1e-6 after the
    binary32 rounding of the estimate); against the FP64 oracle the total
    scatter moves by at most the LUT rounding (2^-11 for F16, 2^-8 for BF16,
    twice for a product) and per-bin errors stay within that bound except in
    the few bins where binary32 and binary64 transport took different
    decisions."""
    from tests import precision
    rep = precision.report(n=400_000)
    say(f"[precision] {rep}")
    bound = {"f32": 1e-6, "f16": 2 * 2.0 ** -11, "bf16": 2 * 2.0 ** -8}
    for name, r in rep["dtypes"].items():
        same = r["vs_fp32_oracle_same_lut"]
        assert r["counts_equal_fp32_oracle"]
        assert same["per_bin_max_rel"] < 1e-6 and same["bins_nonzero_only_in_estimate"] == 0
        ref = r["vs_fp64_oracle_fp32_lut"]
        assert ref["total_scatter_rel"] < bound[name] + 1e-4, (name, ref)
        assert ref["per_bin_median_rel"] <= bound[name] + 1e-6, (name, ref)
