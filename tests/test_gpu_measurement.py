"""Measurement support on the GPU: the per-kernel timing of production
launches (sse_set_kernel_timing / sse_read_kernel_timing) and the device
throughput microbenchmarks (libsse_peaks.so)."""
import ctypes as C
import os

import pytest

from tests import harness as H

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2509_05047_amd as sse  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_kernel_timing_counts_every_production_launch():
    case = H.case_from("tiny")
    ctx, pid = H.open_context(case)
    try:
        with pytest.raises(sse.SseError) as e:
            ctx.read_kernel_timing()
        assert e.value.status == sse.ESTATE
        ctx.set_kernel_timing(True, 2)
        for k in range(3):
            H.run_gpu(ctx, pid, 100_000, 1 + k, stats=False, trues=False)
        t = ctx.read_kernel_timing()
        assert t["launches"] == 2 and t["dropped"] == 1
        assert t["transport_ms"] > 0 and t["coincidence_ms"] > 0
        # instrumented calls are not timed; the count starts again after a read
        H.run_gpu(ctx, pid, 1000, 9, stats=True)
        assert ctx.read_kernel_timing()["launches"] == 0
        ctx.set_kernel_timing(False)
        with pytest.raises(sse.SseError):
            ctx.read_kernel_timing()
    finally:
        ctx.close()


def test_device_peaks_are_plausible():
    lib = C.CDLL(os.path.join(ROOT, "paper_2509_05047_amd", "libsse_peaks.so"))
    import bench
    pk = bench.measure_peaks()
    print(f"[peaks] {pk}", flush=True)
    # Every kind stays below two wave64 instructions per SIMD per 4 cycles
    # at 2.5 GHz (some issue faster than one per 4 cycles on this device)
    ceiling = pk["cus"] * 4 * 16 * 2 * 2.5e9
    for k in ("valu_add", "valu_xor", "valu_fma", "valu_mad64", "valu_cndmask"):
        assert 0.2 * ceiling < pk[k] <= ceiling, (k, pk[k], ceiling)
    assert pk["valu_log"] < 0.5 * pk["valu_add"]   # a transcendental is slower than an add
    assert 0 < pk["sclk_mhz"] < 3000
    assert pk["gather_l2"] > pk["gather_hbm"] > 0
    assert pk["atomic_u32"] > 0 and pk["atomic_f64"] > 0
    assert 1e12 < pk["copy_bytes_per_s"] < 1.2e13
    assert lib is not None
