"""Precision report of the narrow-LUT forms (clinical workload): the final
scatter estimate (scale * W * sens, binary32) computed on the GPU with the
LUT stored in F32, F16 and BF16, against

  * the FP64 oracle: binary64 transport, binary64 accumulation, FP32 LUT
    (the reference the method would give with exact arithmetic and the
    original table), and
  * the binary32 oracle fed the same dequantised LUT (isolates arithmetic:
    the only difference left is the order of the binary64 sums).

Errors are per-bin relative errors over bins nonzero in the reference and
the relative error of the total scatter.  Test infrastructure (it runs the
oracle).
"""
from __future__ import annotations

import numpy as np

import oracle as O
from oracle import post
import workloads as W
from tests import harness as H


def _final(weights, scale, sens_flat):
    return post.apply_sensitivity(weights, scale, sens_flat)


def _errors(est, ref):
    nz = ref != 0
    rel = np.abs(est[nz].astype(np.float64) - ref[nz].astype(np.float64)) / np.abs(ref[nz].astype(np.float64))
    tot_e, tot_r = float(np.sum(est, dtype=np.float64)), float(np.sum(ref, dtype=np.float64))
    extra = int(np.count_nonzero(est[~nz]))
    return {"bins_compared": int(nz.sum()), "per_bin_max_rel": float(rel.max()) if rel.size else 0.0,
            "per_bin_median_rel": float(np.median(rel)) if rel.size else 0.0,
            "per_bin_p99_rel": float(np.quantile(rel, 0.99)) if rel.size else 0.0,
            "bins_nonzero_only_in_estimate": extra,
            "total_scatter_rel": abs(tot_e - tot_r) / abs(tot_r) if tot_r else 0.0}


def report(n=2_000_000, seed=5678, h_offset=0):
    """Run the comparison; returns a dict keyed by LUT dtype name."""
    import torch
    import paper_2509_05047_amd as sse
    base = H.case_from("clinical")
    sens = W.make_sensitivity(base.sino, seed=3, tof_axis=False)
    sens_flat = np.broadcast_to(sens[None], base.sino.shape).reshape(-1)
    scale = post.emission_scale(base.act, base.pdesc.voxel_mm, n)
    # FP64 oracle with the FP32 LUT
    ref64 = H.run_oracle(base, n, seed, h_offset=h_offset, records=False, trues=False, variant="f64")
    ref64_final = _final(ref64["scatter_weights"], scale, sens_flat)
    out = {"histories": n, "reference": "binary64 oracle, FP32 LUT", "dtypes": {}}
    for name, dt in (("f32", sse.F32), ("f16", sse.F16), ("bf16", sse.BF16)):
        case = H.case_from("clinical", lut_dtype=dt)
        ctx, pid = H.open_context(case, sensitivity=sens, sens_tof=False)
        try:
            g = H.run_gpu(ctx, pid, n, seed, h_offset=h_offset, trues=False, stats=False)
            dW = torch.from_numpy(g["scatter_weights"]).cuda()
            fin = torch.empty(case.sino.n_bins, dtype=torch.float32, device="cuda")
            ctx.apply_sensitivity(dW, scale, fin)
            torch.cuda.synchronize()
            est = fin.cpu().numpy()
        finally:
            ctx.close()
        same_lut = H.run_oracle(case, n, seed, h_offset=h_offset, records=False, trues=False)
        same_final = _final(same_lut["scatter_weights"], scale, sens_flat)
        lut_err = np.abs(case.lut.astype(np.float64) - base.lut.astype(np.float64)) / base.lut.astype(np.float64)
        out["dtypes"][name] = {
            "lut_entry_max_rel_rounding": float(lut_err.max()),
            "vs_fp64_oracle_fp32_lut": _errors(est, ref64_final),
            "vs_fp32_oracle_same_lut": _errors(est, same_final),
            "counts_equal_fp32_oracle": bool(np.array_equal(g["scatter_counts"], same_lut["scatter_counts"])),
        }
    return out
