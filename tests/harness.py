"""Shared driver for the parity tests: run the same seeded workload through
the HIP library (via its C ABI binding) and through the CPU oracle, and
compare history by history."""
from __future__ import annotations

import time
from dataclasses import dataclass

import numpy as np

import oracle as O
import workloads as W


@dataclass
class Case:
    scanner: object
    sino: object
    physics: dict
    pdesc: object
    mu: np.ndarray
    act: np.ndarray
    lut_desc: object
    lut: np.ndarray          # float32 values as the oracle sees them
    lut_store: np.ndarray    # values as loaded into the library
    lut_dtype: int = 0
    gaps: dict = None        # gap description (None: plain cylinder)
    edge_t: np.ndarray = None
    edge_a: np.ndarray = None


def with_gaps(case: Case, gaps: dict, policy: str, edge=None, lut_seed=7):
    """The case with the gap model on: the LUT replaced by one with the
    virtual gap indices (values from lut_seed), and for the edge-LUT policy
    the edge LUTs (the oracle's unless `edge` = (transaxial, axial) gives
    them)."""
    dims = W.gap_lut_dims(case.scanner, case.lut_desc.dims)
    ld, vals = W.make_lut(dims, lut_seed, e_min=case.lut_desc.e_min_kev, e_max=case.lut_desc.e_max_kev)
    g = W.gap_desc(gaps, policy)
    et = ea = None
    if policy == "edge_lut":
        if edge is None:
            gt, ga = W.edge_geometries(case.scanner, gaps)
            edge = (O.edge_lut(gt), O.edge_lut(ga))
        et, ea = (np.ascontiguousarray(e, np.float32) for e in edge)
    return Case(case.scanner, case.sino, case.physics, case.pdesc, case.mu, case.act, ld, vals, vals, 0,
                g, et, ea)


def case_from(name, tof_sigma=None, lut_dtype=0, physics=None, phantom=None, lut=None):
    """lut: (LutDesc, float32 values) replacing the workload's own LUT."""
    w = W.WORKLOADS[name]
    pd, mu, act = phantom if phantom is not None else W.make_phantom(w)
    ld, lut = lut if lut is not None else W.make_lut(w.lut_dims, w.lut_seed)
    sino = w.sino if tof_sigma is None else W.Sinogram(**{**w.sino.__dict__, "tof_sigma_mm": tof_sigma})
    store, seen = lut, lut
    if lut_dtype == 1:
        store = lut.astype(np.float16).view(np.uint16)
        seen = lut.astype(np.float16).astype(np.float32)
    elif lut_dtype == 2:
        store = W.to_bf16_bits(lut)
        seen = W.bf16_bits_to_f32(store).reshape(lut.shape)
    return Case(w.scanner, sino, dict(physics or w.physics), pd, mu, act, ld, seen, store, lut_dtype)


def run_gpu(ctx, pid, n, seed, h_offset=0, record_stride=0, trues=True, stream=None, stats=True):
    """stats=False and record_stride=0 run the production (uninstrumented) kernel."""
    import torch
    n_rec = 0 if not record_stride else (n + record_stride - 1) // record_stride
    out = ctx.new_outputs(trues=trues, stats=stats, records=n_rec, record_stride=record_stride or 1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.simulate(pid, n, seed, out, h_offset=h_offset, stream=stream)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    res = {k: (v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in out.items()}
    res["scatter_counts"] = res["scatter_counts"].view(np.uint32)
    if trues:
        res["true_counts"] = res["true_counts"].view(np.uint32)
    if stats:
        res["stats"] = {k: int(v) for k, v in zip(O.ST_NAMES, res["stats"].view(np.uint64))}
    if n_rec:
        res["records"] = np.ascontiguousarray(res["records"]).view(np.uint32).reshape(-1).view(O.RECORD_DTYPE)
    res["seconds"] = dt
    return res


def open_context(case: Case, sensitivity=None, sens_tof=True):
    import paper_2509_05047_amd as sse
    ctx = sse.Context(case.scanner, case.sino, case.physics)
    pid = ctx.load_phantom(case.pdesc, case.mu, case.act)
    ctx.load_lut(case.lut_desc, case.lut_store, dtype=case.lut_dtype)
    if case.gaps is not None:
        ctx.set_gaps(case.gaps, case.edge_t, case.edge_a)
    if sensitivity is not None:
        ctx.load_sensitivity(sensitivity, has_tof_axis=sens_tof)
    return ctx, pid


def run_oracle(case: Case, n, seed, h_offset=0, h_list=None, records=True, trues=True, variant="f32",
               sinograms=True):
    return O.simulate(case.scanner, case.sino, case.physics, case.pdesc, case.mu, activity=case.act,
                      lut_desc=case.lut_desc, lut=case.lut, seed=seed, h0=h_offset, n=n, h_list=h_list,
                      records=records, trues=trues, variant=variant, sinograms=sinograms,
                      gaps=case.gaps, edge_t=case.edge_t, edge_a=case.edge_a)


def record_words(rec):
    return np.ascontiguousarray(rec).view(np.uint32).reshape(len(rec), 32)


def identical_mask(a, b):
    return (record_words(a) == record_words(b)).all(axis=1)


def remove_contributions(counts, weights, rec, which, mask):
    """Subtract the coincidences of the histories selected by mask from a
    (counts, weights) sinogram pair, using their records."""
    c = counts.astype(np.int64).copy()
    w = weights.copy()
    sel = rec[mask]
    sel = sel[(sel["outcome"] & 0xFF) == which]
    b = O.record_bins(sel)
    np.subtract.at(c, b, 1)
    np.subtract.at(w, b, sel["weight"].astype(np.float64))
    return c, w


def compare_sinograms(gpu, orc, g_rec, o_rec, same, rel_tol=1e-5):
    """Counts of the identical histories bit-exact, weights within rel_tol
    per bin, zero where the oracle is zero.  Returns the max relative weight
    difference over nonzero bins."""
    worst = 0.0
    for which, cname, wname in ((0, "scatter_counts", "scatter_weights"), (1, "true_counts", "true_weights")):
        if gpu.get(cname) is None or orc.get(cname) is None:
            continue
        gc, gw = remove_contributions(gpu[cname], gpu[wname], g_rec, which, ~same)
        oc, ow = remove_contributions(orc[cname], orc[wname], o_rec, which, ~same)
        assert np.array_equal(gc, oc), f"{cname}: {np.count_nonzero(gc != oc)} bins differ"
        nz = ow != 0
        assert np.all(gw[~nz] == 0.0)
        if nz.any():
            rel = np.abs(gw[nz] - ow[nz]) / np.abs(ow[nz])
            worst = max(worst, float(rel.max()))
            assert rel.max() <= rel_tol, (wname, rel.max())
    return worst


def describe_mismatch(g, o, limit=3):
    gw, ow = record_words(g), record_words(o)
    bad = np.nonzero((gw != ow).any(1))[0]
    lines = []
    for i in bad[:limit]:
        cols = np.nonzero(gw[i] != ow[i])[0]
        lines.append(f"record {i}: words {cols.tolist()} gpu {gw[i][cols].tolist()} oracle {ow[i][cols].tolist()}")
    return "\n".join(lines)
