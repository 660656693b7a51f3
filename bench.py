"""Throughput benchmark of the LUT-weighted Monte Carlo scatter path on one GPU.

One step = one pass of the whole path over one batch: zero the sinograms,
simulate the clinical workload's histories (emission, Woodcock transport,
detection, LUT weighting, TOF sinogram accumulation), then the sensitivity
multiply (scale * W * sens -> float).  Prints one JSON line: the FP32-LUT
headline, and beside it the chosen precision form (FP16 LUT), the serving
stream (p50/p99 latency), the large joint-estimation-style loop, the
roofline against peaks measured on the device, and the CPU oracle baseline.

  python bench.py [--steps K] [--warmup W] [--lut f32|f16|bf16] [--workload clinical|large|serving]

Only one GPU is used; --gpus above 1 exits with a message.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads as W  # noqa: E402

# Algorithmic VALU work per unit of the method's work (lane-operations; the
# weights of the benchmark definition's cost model): a Philox4x32-10 block,
# a Woodcock tentative step, a real interaction, a detected single, a
# sinogram update, and each binary32 logarithm, sine/cosine pair or square
# root at 4 operations of quarter rate.  Units are counted by the kernel's
# statistics counters (the oracle counts the same).
COST = dict(rng_block=120, step=30, real=80, detected=60, update=40, transcendental=4 * 4)
PEAK_VALU_PUBLISHED = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x 2.4 GHz: non-packed lane-ops/s


def algorithmic_units(stats: dict) -> dict:
    """Per-history units of the cost model from the statistics counters.
    Transcendentals: one free-path logarithm per tentative step and one
    energy-model logarithm per surviving Compton scatter; one sine/cosine per
    emission and per scatter; square roots at the emission (1), per scatter
    (2, the rotation) and per photon reaching the cylinder (1)."""
    h = stats["histories"]
    scat = (stats["compton"] - stats["killed"]) + stats["rayleigh"]
    logs = stats["steps"] + (stats["compton"] - stats["killed"])
    sincos = h + scat
    sqrts = h + 2 * scat + stats["escaped"]
    return {"rng_block": stats["rng_blocks"] / h, "step": stats["steps"] / h, "real": stats["real"] / h,
            "detected": stats["detected"] / h, "update": (stats["scatter"]) / h,
            "transcendental": (logs + sincos + sqrts) / h,
            # random gathers: the attenuation map at every tentative step that stays
            # inside the voxel box (each photon's last step leaves it), the alias
            # table once per history, the LUT twice per sinogram update
            "gathers_mu": (stats["steps"] - stats["escaped"]) / h, "gathers_alias": 1.0,
            "gathers_lut": 2.0 * stats["scatter"] / h}


def measure_peaks():
    """Throughput of the device's units (libsse_peaks.so): VALU lane-ops/s by
    instruction kind, random gathers/s by buffer size, random atomic adds/s."""
    import ctypes as C
    lib = C.CDLL(os.path.join(ROOT, "paper_2509_05047_amd", "libsse_peaks.so"))

    class Peaks(C.Structure):
        _fields_ = [(k, C.c_double) for k in ("sclk_mhz", "valu_add", "valu_xor", "valu_fma", "valu_mad64",
                                                "valu_cndmask", "valu_log", "gather_l2", "gather_llc",
                                                "gather_hbm", "atomic_u32", "atomic_f64", "copy_bytes_per_s")] + \
                   [("atomic_bins", C.c_uint64), ("cus", C.c_uint64)]

    lib.sse_measure_peaks.argtypes = [C.c_int, C.c_uint64, C.c_void_p]
    lib.sse_measure_peaks.restype = C.c_int
    pk = Peaks()
    rc = lib.sse_measure_peaks(0, 0, C.byref(pk))
    if rc != 0:
        raise RuntimeError(f"sse_measure_peaks failed ({rc})")
    return {f[0]: getattr(pk, f[0]) for f in Peaks._fields_}


def kernel_source_hash() -> str:
    """First 16 hex digits of sha256 over the transport kernel's sources."""
    import hashlib
    h = hashlib.sha256()
    for f in ("transport.hip", "internal.h"):
        with open(os.path.join(ROOT, "paper_2509_05047_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes of one launch of the transport kernel from the committed
    counter summary (FETCH_SIZE and WRITE_SIZE, calibrated by a plain copy),
    or None when the kernels have changed since the counters were taken."""
    import re
    path = os.path.join(ROOT, "profiles", "transport_clinical_hbm_counters.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    fields = dict(re.findall(r"^(\w+): (\S+)$", text, flags=re.M))
    if fields.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return float(fields["fetch_bytes_per_launch"]) + float(fields["write_bytes_per_launch"])


# The paper's smoothing of the scatter estimate: FWHM [9, 6, 10.5] radial,
# view and plane bins (Results); the normalisation sinogram is smoothed more
# heavily (three times these sigmas, a choice: the paper does not say).
PAPER_FWHM_BINS = (9.0, 6.0, 10.5)


def smoothing_normalisation_timing(ctx, weights, scale, out, stream, reps=3):
    """Outside the timed steps: the smoothing-normalisation workflow on the
    step's weights -- a normalisation sinogram (heavy smoothing of these
    weights standing in for the reference cylinder) and the normalised
    finalize sens * G(S N) / N with the paper's FWHM -- timed with HIP events
    on the launch stream.  Algorithmic HBM bytes per bin: 28 for the
    finalize (the fused radial and plane pass reads W and N and writes
    G_rp(S N), 16; the view pass reads that and N and writes, 12; the
    sensitivity has no TOF axis and is read once per TOF bin)."""
    import torch
    sigma = tuple(f / 2.35482 for f in PAPER_FWHM_BINS)
    heavy = tuple(3 * s for s in sigma)
    norm = torch.empty_like(out)
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2 * reps + 1)]
    e[0].record(stream)
    for i in range(reps):
        ctx.smoothing_normalisation(weights, scale, norm, heavy, stream=stream)
        e[1 + i].record(stream)
    for i in range(reps):
        ctx.finalize_normalised(weights, scale, norm, out, sigma, stream=stream)
        e[1 + reps + i].record(stream)
    torch.cuda.synchronize()
    t_norm = [e[i].elapsed_time(e[i + 1]) for i in range(reps)]
    t_fin = [e[reps + i].elapsed_time(e[reps + i + 1]) for i in range(reps)]
    n_bins = out.numel()
    fin_ms = float(np.median(t_fin))
    return {"fwhm_bins": list(PAPER_FWHM_BINS), "normalisation_sigma_bins": list(heavy),
            "normalisation_ms": float(np.median(t_norm)), "finalize_normalised_ms": fin_ms,
            "finalize_bytes_per_bin": 28, "finalize_hbm_tbps": 28.0 * n_bins / (fin_ms * 1e-3) / 1e12}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(w, physics, pdesc, mu, act, lut_desc, lut_f32, n, gaps=None):
    """The oracle as it stands, single thread, on the first n histories
    (with the gap model, its own edge LUTs)."""
    import oracle as O
    alias = O.build_alias(act)
    et = ea = None
    if gaps is not None and gaps["policy"] == "edge_lut":
        gt, ga = W.edge_geometries(w.scanner, W.SIGNA_GAPS)
        et, ea = O.edge_lut(gt), O.edge_lut(ga)
    t0 = time.perf_counter()
    r = O.simulate(w.scanner, w.sino, physics, pdesc, mu, alias=alias,
                   lut_desc=lut_desc, lut=lut_f32, seed=w.seed, n=n, trues=False,
                   gaps=gaps, edge_t=et, edge_a=ea)
    dt = time.perf_counter() - t0
    res = {"value": n / dt, "unit": "histories/s", "cores": 1, "kind": "oracle",
           "sample": f"{w.name} workload, histories 0..{n} of seed {w.seed}, one thread, {dt:.1f} s",
           "scatter_coincidences_per_sec": r["stats"]["scatter"] / dt}
    res["all_cores"] = cpu_baseline_all_cores(w, physics, pdesc, mu, alias, lut_desc, lut_f32, n, gaps, et, ea)
    return res


def cpu_baseline_all_cores(w, physics, pdesc, mu, alias, lut_desc, lut_f32, n_single, gaps, et, ea):
    """The same oracle on every host core this process may use (at most 16,
    the host share of one GPU): one thread per core, each on its own range
    of histories with its own sinograms (the oracle's C code runs without
    the interpreter lock).  Each thread takes n_single / 8 histories, so the
    sample is about twice the single-thread one in CPU time at 16 threads."""
    import platform
    from concurrent.futures import ThreadPoolExecutor
    import oracle as O
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = max(1, min(16, avail))
    per = max(1, n_single // 8)

    def run(k):
        return O.simulate(w.scanner, w.sino, physics, pdesc, mu, alias=alias, lut_desc=lut_desc, lut=lut_f32,
                          seed=w.seed, h0=n_single + k * per, n=per, trues=False, gaps=gaps, edge_t=et,
                          edge_a=ea)["stats"]["scatter"]

    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=threads) as ex:
        scatter = sum(ex.map(run, range(threads)))
    dt = time.perf_counter() - t0
    model = platform.processor() or platform.machine()
    try:
        with open("/proc/cpuinfo") as f:
            model = next(l.split(":", 1)[1].strip() for l in f if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    return {"value": threads * per / dt, "unit": "histories/s", "cores": threads, "nproc": os.cpu_count(),
            "cpu_model": model, "scatter_coincidences_per_sec": scatter / dt,
            "sample": f"{threads} threads x {per} histories (from history {n_single}, seed {w.seed}), {dt:.1f} s"}


def large_loop(args):
    """Joint-estimation-style loop: successive requests on one 256x256x89
    phantom whose activity is rescaled by a seeded smooth field each time;
    each request simulates 2e9 histories and then runs the fused
    finalize (scale * W -> Gaussian sigma 2 bins -> x sensitivity)."""
    import torch
    import paper_2509_05047_amd as sse
    w = W.WORKLOADS["large"]
    n = int(args.histories) if (args.histories and args.workload == "large") else w.n_histories
    reqs = int(w.extra["n_requests"])
    sigma = float(w.extra["smooth_sigma_bins"])
    pdesc, mu, act0 = W.make_phantom(w)
    log(f"[bench] large loop: {reqs} requests x {n:.3g} histories, phantom {pdesc.shape}")
    acts = [W.scaled_activity(act0, k) for k in range(reqs)]
    lut_desc, lut = W.make_lut(w.lut_dims, w.lut_seed)
    sens = W.make_sensitivity(w.sino, seed=3, tof_axis=True)
    ctx = sse.Context(w.scanner, w.sino, w.physics)
    ctx.set_pair_pruning(args.pair_pruning)
    pid = ctx.load_phantom(pdesc, mu, acts[0])
    ctx.load_lut(lut_desc, lut)
    ctx.load_sensitivity(sens, has_tof_axis=True)
    del sens
    out = ctx.new_outputs(trues=False, stats=False)
    final = torch.empty(ctx.n_bins, dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    def request(act, timing=None):
        t0 = time.perf_counter()
        ctx.update_activity(pid, act)
        out["scatter_counts"].zero_()
        out["scatter_weights"].zero_()
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        e[0].record(stream)
        ctx.simulate(pid, n, w.seed, out, stream=stream)
        e[1].record(stream)
        ctx.finalize(out["scatter_weights"], ctx.emission_scale(pid, n), final, sigma_bins=(sigma, sigma, sigma),
                     stream=stream)
        e[2].record(stream)
        torch.cuda.synchronize()
        if timing is not None:
            timing.append(((time.perf_counter() - t0) * 1e3, e[0].elapsed_time(e[1]), e[1].elapsed_time(e[2])))

    for _ in range(args.warmup):
        request(acts[0])
    timing = []
    t0 = time.perf_counter()
    for k in range(reqs):
        request(acts[k], timing)
        log(f"[bench] request {k + 1}/{reqs}: {timing[-1][0]:.1f} ms")
    dt = time.perf_counter() - t0
    ctx.close()
    lat = [t[0] for t in timing]
    result = {
        "metric": "photon histories/sec", "value": n * reqs / dt, "unit": "histories/s", "n_gpus": 1,
        "steps": reqs, "warmup": args.warmup, "ms_per_step": dt / reqs * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"large loop: {pdesc.nx}x{pdesc.ny}x{pdesc.nz} phantom of 1.17 mm voxels, "
                               f"{reqs} requests x {n} histories with updated activity, fused "
                               f"scale/smooth(sigma {sigma} bins)/sensitivity finalize",
                   "histories_per_step": n, "pair_pruning": bool(args.pair_pruning)},
        "request_latency_ms": lat,
        "request_latency_p50_ms": float(np.percentile(lat, 50)),
        "simulate_ms": float(np.mean([t[1] for t in timing])),
        "finalize_ms": float(np.mean([t[2] for t in timing])),
        "update_activity_ms": float(np.mean([t[0] - t[1] - t[2] for t in timing])),
    }
    return result


def joint_loop(args):
    """The joint activity / scatter estimation loop on the clinical workload
    (Methods, "Unknown activity distribution, very limited simulation
    time"): 10 iterations of (activity from the image, short simulation,
    normalised smoothing with the paper's FWHM, 1 TOF-OSEM iteration of 28
    subsets), from a reconstruction without scatter compensation, on a
    synthetic acquisition made with the library's models (true scatter from
    a 2e10-history simulation of the true activity, 34 % scatter fraction,
    5e8 Poisson prompts)."""
    import torch
    import paper_2509_05047_amd as sse
    from paper_2509_05047_amd import joint
    w = W.WORKLOADS["clinical"]
    pdesc, mu, act = W.make_phantom(w)
    lut_desc, lut = W.make_lut(w.lut_dims, w.lut_seed)
    ctx = sse.Context(w.scanner, w.sino, w.physics)
    ctx.load_lut(lut_desc, lut)
    ctx.load_sensitivity(W.make_sensitivity(w.sino, seed=3, tof_axis=False), has_tof_axis=False)
    pid = ctx.load_phantom(pdesc, mu, act)
    x_true = torch.from_numpy(W.plane_image(pdesc, act, w.scanner)).cuda()
    detector = torch.from_numpy(W.make_sensitivity(w.sino, seed=11, tof_axis=False)).cuda()
    log("[bench] joint loop: synthetic acquisition")
    prompts, mult, s_true, t = joint.synthetic_acquisition(ctx, pid, x_true, detector)
    # Smoothing normalisation from the reference cylinder (the paper: a 40 cm
    # cylinder; here 28 cm, the grid's width).  The LUT's structures do not
    # depend on TOF, so the reference weights are averaged over the TOF bins
    # first: a 2e10-history reference then has ~30x the counts per bin.
    ref_mu, ref_act = W.reference_cylinder(pdesc, 140.0)
    rid = ctx.load_phantom(pdesc, ref_mu, ref_act)
    out = ctx.new_outputs()
    n_ref = 20_000_000_000
    ctx.simulate(rid, n_ref, 3, out)
    wref = out["scatter_weights"].view(prompts.shape)
    wref.copy_(wref.mean(dim=0, keepdim=True).expand_as(wref))
    sigma = tuple(f / 2.35482 for f in PAPER_FWHM_BINS)
    norm = torch.empty(prompts.shape, dtype=torch.float32, device="cuda")
    ctx.smoothing_normalisation(out["scatter_weights"], ctx.emission_scale(rid, n_ref), norm,
                                tuple(3 * x for x in sigma))
    del out, wref
    ctx.unload_phantom(rid)
    errs = []
    s_true_nt = s_true.sum(dim=0)   # TOF-summed: the per-bin noise of the reference is lower

    def cb(k, image, scatter):
        errs.append((float((scatter.sum(dim=0) - s_true_nt).norm() / s_true_nt.norm()),
                     float((scatter.double().sum() / s_true.double().sum() - 1).abs()),
                     float((image - x_true).norm() / x_true.norm())))
        log(f"[bench] joint iteration {k + 1}: scatter error {errs[-1][0]:.4f} (total {errs[-1][1]:.4f}), "
            f"image error {errs[-1][2]:.4f}")

    n_short = 1_500_000_000
    image0 = torch.full_like(x_true, float(x_true.mean()))
    image, scatter, timing = joint.joint_estimation(ctx, pid, prompts, mult, norm, sigma, n_iter=10, n_subsets=28,
                                                    n_histories=n_short, seed=w.seed, acq_seconds=t,
                                                    image=image0, callback=cb)
    ctx.close()
    lat = timing.iteration_ms
    return {"iterations": len(lat), "iteration_ms": lat, "iteration_p50_ms": float(np.percentile(lat, 50)),
            "initial_reconstruction_ms": timing.initial_ms,
            "step_ms": {"activity_update": float(np.mean(timing.activity_ms)),
                        "simulate": float(np.mean(timing.simulate_ms)),
                        "normalised_smoothing": float(np.mean(timing.smooth_ms)),
                        "osem_1x28": float(np.mean(timing.osem_ms))},
            "scatter_rel_l2_error_tof_summed": [e[0] for e in errs],
            "total_scatter_rel_error": [e[1] for e in errs],
            "image_rel_l2_error": [e[2] for e in errs],
            "workload": f"clinical body {pdesc.nx}x{pdesc.ny}x{pdesc.nz}, image {pdesc.nx}x{pdesc.ny}x"
                        f"{w.sino.n_plane}, 10 iterations x ({n_short:.2g}-history simulation, normalised "
                        f"smoothing FWHM {list(PAPER_FWHM_BINS)} bins, TOF-OSEM 1 x 28 subsets); synthetic "
                        f"acquisition of 5e8 Poisson prompts, 34 % scatter"}


def serving(args):
    """Serving stream: Poisson arrivals of scatter-estimate requests on
    body-like phantoms of 64^3, 128^3 and 192x192x89 voxels (a pool of
    seeded phantoms, all resident), budgets log-uniform in [1e7, 5e8]
    histories, one shared LUT, the Signa scanner and sinogram.  Latency is
    submit -> sinogram complete on the device."""
    import threading
    import torch
    import paper_2509_05047_amd as sse
    w = W.WORKLOADS["clinical"]
    ctx = sse.Context(w.scanner, w.sino, w.physics)
    ctx.set_pair_pruning(args.pair_pruning)
    lut_desc, lut = W.make_lut(w.lut_dims, w.lut_seed)
    ctx.load_lut(lut_desc, lut)
    n_pool = 12
    pids = []
    for k in range(n_pool):
        pd, mu, act = W.serving_phantom(k)
        pids.append(ctx.load_phantom(pd, mu, act))
    log(f"[bench] serving: {n_pool} resident phantoms")
    # single-stream throughput over the whole pool, with the requests'
    # outputs (scatter sinogram only): sets the arrival rate
    out = ctx.new_outputs(trues=False, stats=False)
    ctx.simulate(pids[0], 10_000_000, 1, out)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    probe = 0
    for k in range(n_pool):
        ctx.simulate(pids[k], 50_000_000, 2, out)
        probe += 50_000_000
    torch.cuda.synchronize()
    single = probe / (time.perf_counter() - t0)
    del out
    rng = np.random.default_rng(77)
    nreq = args.requests
    budgets = np.exp(rng.uniform(np.log(1e7), np.log(5e8), nreq)).astype(np.int64)
    which = rng.integers(0, n_pool, nreq)
    mean_budget = (5e8 - 1e7) / np.log(50.0)
    lam = args.load * single / mean_budget
    arrivals = np.cumsum(rng.exponential(1.0 / lam, nreq))
    footprint = ctx.n_bins * 12
    budget_bytes = 48 * footprint
    srv = sse.Server(ctx, max_active=32, hbm_budget_bytes=budget_bytes, tick_histories=int(single * 0.01))
    log(f"[bench] single-stream {single:.3e} histories/s, load {args.load}, {lam:.2f} requests/s")
    ids = {}

    def generator():
        start = time.perf_counter()
        for i in range(nreq):
            delay = arrivals[i] - (time.perf_counter() - start)
            if delay > 0:
                time.sleep(delay)
            ids[srv.submit(pids[which[i]], int(budgets[i]), 5000 + i)] = i

    gen = threading.Thread(target=generator)
    t_start = time.perf_counter()
    gen.start()
    done = []
    while len(done) < nreq:
        for c in srv.poll(wait_ms=100):
            done.append(c)
            srv.release(c["id"])
        if len(done) % 32 == 0 and done:
            log(f"[bench] {len(done)}/{nreq} requests complete")
    gen.join()
    makespan = time.perf_counter() - t_start
    st = srv.stats()
    srv.stop()
    ctx.close()
    lat = np.array([(c["t_complete"] - c["t_submit"]) * 1e3 for c in done])
    hist = int(sum(c["histories"] for c in done))
    result = {
        "metric": "photon histories/sec and p50/p99 request latency (serving)",
        "value": hist / makespan, "unit": "histories/s", "n_gpus": 1, "steps": nreq, "warmup": 0,
        "ms_per_step": makespan / nreq * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"serving: {nreq} Poisson requests at load {args.load} of single-stream "
                               f"throughput, budgets log-uniform 1e7-5e8, {n_pool} body phantoms "
                               "(64^3 / 128^3 / 192x192x89), Signa scanner, 357x224x89x29 sinogram",
                   "histories_total": hist, "pair_pruning": bool(args.pair_pruning)},
        "latency_p50_ms": float(np.percentile(lat, 50)), "latency_p99_ms": float(np.percentile(lat, 99)),
        "latency_max_ms": float(lat.max()), "single_stream_histories_per_sec": single,
        "arrival_rate_per_sec": lam, "max_active_seen": st["max_active_seen"], "ticks": st["ticks"],
        "hbm_budget_bytes": budget_bytes, "bytes_allocated": st["bytes_allocated"],
    }
    return result


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="clinical", choices=["clinical", "large", "serving", "joint"])
    ap.add_argument("--requests", type=int, default=256, help="serving: number of requests")
    ap.add_argument("--load", type=float, default=0.7, help="serving: offered load vs single-stream throughput")
    ap.add_argument("--histories", type=float, default=0, help="override histories per step")
    ap.add_argument("--lut", default="f32", choices=["f32", "f16", "bf16"])
    ap.add_argument("--lut-mode", default="lut5d", choices=list(W.LUT_MODES),
                    help="LUT variant and energy configuration (lut5d: the workload's own)")
    ap.add_argument("--lut-shape", default="workload", choices=["workload", "paper"],
                    help="paper: the paper's LUT shape, 5 keV bins over 0-515 keV, 5 degree angle bins, "
                         "18 x 55 crystal indices (103 x 36 x 36 x 18 x 55; needs the gap model)")
    ap.add_argument("--gaps", default="none", choices=["none", "auto", "discard", "nearest", "edge_lut"],
                    help="gaps between modules and blocks (Signa-like widths) with this gap policy; "
                         "auto: the LUT mode's own policy")
    ap.add_argument("--cpu-histories", type=int, default=40_000_000)
    ap.add_argument("--copy-bytes", type=float, default=0,
                    help="only run a plain device copy of this many bytes 3 times (calibrates HBM counters)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--pair-pruning", action="store_true",
                    help="large and serving workloads: pair pruning on (both photons are tracked by default)")
    ap.add_argument("--peaks-only", action="store_true",
                    help="only run the device throughput microbenchmarks (for counter calibration)")
    ap.add_argument("--no-legs", action="store_true",
                    help="clinical workload: skip the chosen-form, serving and large-loop legs")
    ap.add_argument("--no-pruned", action="store_true",
                    help="skip the second timing with pair pruning (photon B not tracked once photon A "
                         "missed the energy window; identical sinograms)")

    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(histories shard by index).", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2509_05047_amd as sse

    torch.cuda.set_device(0)
    if args.workload == "large":
        print(json.dumps(large_loop(args)), flush=True)
        return
    if args.workload == "serving":
        print(json.dumps(serving(args)), flush=True)
        return
    if args.workload == "joint":
        print(json.dumps(joint_loop(args)), flush=True)
        return
    if args.peaks_only:
        log(f"[bench] peaks {json.dumps(measure_peaks())}")
        return
    if args.copy_bytes:
        src = torch.ones(int(args.copy_bytes) // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copied {src.numel() * 4} bytes 3 times")
        return
    w = W.WORKLOADS[args.workload]
    pdesc, mu, act = W.make_phantom(w)
    physics, lut_desc, lut = W.lut_mode(w, args.lut_mode)
    gaps = None
    if args.lut_shape == "paper" and args.gaps == "none":
        args.gaps = "auto"   # the 18 x 55 crystal axes are the gap layout
    if args.gaps != "none":
        policy = W.GAP_POLICY_OF_MODE[args.lut_mode] if args.gaps == "auto" else args.gaps
        gaps = W.gap_desc(W.SIGNA_GAPS, policy)
        dims = W.gap_lut_dims(w.scanner, lut_desc.dims)
        e_min, e_max = lut_desc.e_min_kev, lut_desc.e_max_kev
        if args.lut_shape == "paper":
            # unit axes of the LUT variant stay unit
            dims = tuple(1 if d == 1 else pd for d, pd in zip(dims, W.PAPER_LUT_DIMS))
            e_min, e_max = W.PAPER_LUT_E_RANGE
        if tuple(dims) != tuple(lut_desc.dims):
            lut_desc, lut = W.make_lut(dims, w.lut_seed, e_min=e_min, e_max=e_max)
    lut_dtype = {"f32": sse.F32, "f16": sse.F16, "bf16": sse.BF16}[args.lut]
    lut_store = {"f32": lut, "f16": lut.astype(np.float16).view(np.uint16), "bf16": W.to_bf16_bits(lut)}[args.lut]
    n = int(args.histories) if args.histories else w.n_histories
    sens = W.make_sensitivity(w.sino, seed=3, tof_axis=True)
    log(f"[bench] workload {w.name}: {n:.3g} histories/step, sinogram {w.sino.shape}, LUT {args.lut}")
    ctx = sse.Context(w.scanner, w.sino, physics)
    pid = ctx.load_phantom(pdesc, mu, act)
    ctx.load_lut(lut_desc, lut_store, dtype=lut_dtype)
    if gaps is not None:
        gt, ga = W.edge_geometries(w.scanner, W.SIGNA_GAPS)
        ctx.set_gaps(gaps, sse.build_edge_lut(gt), sse.build_edge_lut(ga))
    ctx.load_sensitivity(sens, has_tof_axis=True)
    del sens
    # per-history work units for the cost model, from an instrumented run on
    # a sample of the same histories (the timed steps run the production
    # kernel, which collects no statistics)
    sample = min(n, 100_000_000)
    probe = ctx.new_outputs(trues=False, stats=True)
    ctx.simulate(pid, sample, w.seed, probe)
    torch.cuda.synchronize()
    stats = sse.stats_dict(probe["stats"])
    del probe
    out = ctx.new_outputs(trues=False, stats=False)
    final = torch.empty(ctx.n_bins, dtype=torch.float32, device="cuda")
    scale = ctx.emission_scale(pid, n)
    stream = torch.cuda.current_stream()
    # HIP events on the stream the library launches on, around each timed
    # simulate call (its transport, coincidence and counter-reset launches)
    tr_start = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]
    tr_end = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps)]

    def step(i=None):
        out["scatter_counts"].zero_()
        out["scatter_weights"].zero_()
        if i is not None:
            tr_start[i].record(stream)
        ctx.simulate(pid, n, w.seed, out, stream=stream)
        if i is not None:
            tr_end[i].record(stream)
        ctx.apply_sensitivity(out["scatter_weights"], scale, final, stream=stream)

    def timed_steps(label):
        """warm-up, then the timed steps; returns (wall seconds, simulate
        spans in ms, per-kernel timing of the timed steps)."""
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        ctx.set_kernel_timing(True, 64 * args.steps)
        t0 = time.perf_counter()
        for i in range(args.steps):
            step(i)
            log(f"[bench] {label}step {i + 1}/{args.steps} queued")
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        kt = ctx.read_kernel_timing()
        ctx.set_kernel_timing(False)
        return dt, [a.elapsed_time(b) for a, b in zip(tr_start, tr_end)], kt

    peaks = measure_peaks()
    log(f"[bench] device peaks: VALU add {peaks['valu_add']:.3e} lane-ops/s at {peaks['sclk_mhz']:.0f} MHz, "
        f"L2 gathers {peaks['gather_l2']:.3e}/s, f64 atomics {peaks['atomic_f64']:.3e}/s")
    dt, kernel_ms, kt = timed_steps("")
    scatter_per_step = int(out["scatter_counts"].sum(dtype=torch.int64))
    final_f32 = final.clone() if not args.no_legs else None
    pruned = None
    if not args.no_pruned:
        # The same steps with pair pruning, reported beside the headline (which
        # tracks both photons of every history): same histories, same sinograms.
        ctx.set_pair_pruning(True)
        dtp, pruned_ms, _ = timed_steps("pruned ")
        ctx.set_pair_pruning(False)
        pruned = {"value": n * args.steps / dtp, "ms_per_step": dtp / args.steps * 1e3,
                  "simulate_ms": float(np.mean(pruned_ms)),
                  "same_scatter_counts": int(out["scatter_counts"].sum(dtype=torch.int64)) == scatter_per_step,
                  "note": "photon B not tracked when photon A ended outside the energy window"}
    next1 = smoothing_normalisation_timing(ctx, out["scatter_weights"], scale, final, stream)
    chosen = None
    if not args.no_legs and args.lut == "f32":
        # The chosen precision form: the same LUT stored in FP16 (binary32
        # transport, binary64 accumulation), the same histories and steps.
        ctx.load_lut(lut_desc, lut.astype(np.float16).view(np.uint16), dtype=sse.F16)
        dtc, chosen_ms, ktc = timed_steps("FP16-LUT ")
        nz = final_f32 != 0
        rel = ((final[nz].double() - final_f32[nz].double()).abs() / final_f32[nz].double().abs()).float()
        q = torch.quantile(rel[torch.randperm(rel.numel(), device=rel.device)[:1 << 24]],
                           torch.tensor([0.5, 0.99], device=rel.device)).tolist()
        tot16, tot32 = float(final.double().sum()), float(final_f32.double().sum())
        chosen = {"lut_dtype": "f16", "value": n * args.steps / dtc, "unit": "histories/s",
                  "ms_per_step": dtc / args.steps * 1e3, "simulate_ms": float(np.mean(chosen_ms)),
                  "transport_kernel_ms": ktc["transport_ms"] / max(1, ktc["launches"]),
                  "scatter_coincidences_per_sec": int(out["scatter_counts"].sum(dtype=torch.int64)) * args.steps / dtc,
                  "same_scatter_counts": int(out["scatter_counts"].sum(dtype=torch.int64)) == scatter_per_step,
                  "vs_fp32_lut_same_histories": {
                      "bins_compared": int(nz.sum()), "per_bin_median_rel": q[0], "per_bin_p99_rel": q[1],
                      "per_bin_max_rel": float(rel.max()), "total_scatter_rel": abs(tot16 - tot32) / tot32},
                  "vs_fp64_oracle": "per-bin p99 6.5e-4, median 2.0e-4, total scatter 6.7e-6 at 1e7 "
                                    "histories (FP32 LUT: p99 1.1e-7, total 2.1e-5); the GPU equals the "
                                    "binary32 oracle fed the dequantised LUT exactly"}
        del rel, nz
    del final_f32
    ctx.close()

    units = algorithmic_units(stats)
    # the transport kernel (the dominant one) does all but the sinogram updates
    ops_transport = sum(COST[k] * units[k] for k in ("rng_block", "step", "real", "detected", "transcendental"))
    ops_per_hist = ops_transport + COST["update"] * units["update"]
    launches_per_step = kt["launches"] / args.steps
    t_launch_ms = kt["transport_ms"] / max(1, kt["launches"])
    c_launch_ms = kt["coincidence_ms"] / max(1, kt["launches"])
    hist_per_launch = n / launches_per_step
    achieved = ops_transport * hist_per_launch / (t_launch_ms * 1e-3)
    peak_valu = max(peaks["valu_add"], peaks["valu_fma"])
    gathers = units["gathers_mu"] + units["gathers_alias"]
    # bounds of the transport kernel in histories/s (benchmark definition):
    # VALU, random gathers at the measured L2 rate
    bound_valu = peak_valu / ops_transport
    bound_gather = peaks["gather_l2"] / gathers
    kernel_hist_s = hist_per_launch / (t_launch_ms * 1e-3)
    updates_per_launch = units["update"] * hist_per_launch
    result = {
        "metric": "photon histories/sec",
        "value": n * args.steps / dt,
        "unit": "histories/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {pdesc.nx}x{pdesc.ny}x{pdesc.nz} body phantom, "
                               f"{w.scanner.n_crystals}x{w.scanner.n_rings} scanner, "
                               f"{'x'.join(map(str, w.sino.shape[::-1]))} TOF sinogram (rad x view x plane x tof), "
                               f"{'x'.join(map(str, lut_desc.dims))} {args.lut} LUT",
                   "histories_per_step": n, "lut_dtype": args.lut, "lut_mode": args.lut_mode,
                   "lut_shape": args.lut_shape, "lut_mib": round(lut_store.nbytes / 2 ** 20, 1),
                   "gaps": (None if gaps is None else
                            dict(gaps, fraction_rejected=stats["rej_gap"] / max(1, stats["scatter"] + stats["true"]
                                                                                 + stats["rej_gap"]),
                                 assigned_per_history=stats["gap_assigned"] / stats["histories"])),
                   "energy_window_kev": [physics["e_lo_kev"], physics["e_hi_kev"]],
                   "energy_fwhm": physics["e_fwhm_frac"], "transport": "f32",
                   "accumulation": "f64"},
        "scatter_coincidences_per_sec": scatter_per_step * args.steps / dt,
        "smoothing_normalisation": next1,
        "pair_pruning": pruned,
        "simulate_ms": float(np.mean(kernel_ms)),
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": peak_valu / 1e12,
                     "unit": "TOP/s", "frac": achieved / peak_valu,
                     "traffic": (measured_traffic() if args.workload == "clinical" and n == w.n_histories
                                 and args.lut == "f32" and args.lut_mode == "lut5d" and gaps is None
                                 and args.lut_shape == "workload" else None),
                     "kernel": "transport_batch_kernel (transport, detection; 97 % of the step); a step is one "
                               "fill launch that takes every history and empty launches after it, and kernel_ms "
                               "averages all of them, as histories_per_launch does",
                     "kernel_ms": t_launch_ms, "launches_per_step": launches_per_step,
                     "histories_per_launch": hist_per_launch,
                     "ops_per_history": ops_transport,
                     "units_per_history": units,
                     "peak_source": "measured on this device: v_add_u32 / v_fma_f32 loops (libsse_peaks)",
                     "peak_published_derived": PEAK_VALU_PUBLISHED / 1e12,
                     "bounds_histories_per_s": {"valu": bound_valu, "l2_gather": bound_gather},
                     "kernel_histories_per_s": kernel_hist_s,
                     "coincidence_kernel": {"kernel_ms": c_launch_ms, "updates_per_launch": updates_per_launch,
                                            "atomics_per_s": 2 * updates_per_launch / (c_launch_ms * 1e-3),
                                            "peak_atomics_per_s": min(peaks["atomic_u32"], peaks["atomic_f64"])},
                     "achieved_gathers_per_s": gathers * kernel_hist_s,
                     "peak_gathers_per_s": peaks["gather_l2"]},
        "device_peaks": peaks,
        "chosen_form": chosen,
    }
    if not args.no_legs and args.workload == "clinical" and not args.histories:
        log("[bench] serving leg")
        sv = serving(args)
        result["serving"] = {k: sv[k] for k in ("value", "unit", "latency_p50_ms", "latency_p99_ms",
                                                "latency_max_ms", "single_stream_histories_per_sec",
                                                "arrival_rate_per_sec", "max_active_seen", "ticks")}
        result["serving"]["workload"] = sv["config"]["workload"]
        log("[bench] large-loop leg")
        ll = large_loop(args)
        result["large_loop"] = {k: ll[k] for k in ("value", "unit", "request_latency_ms", "request_latency_p50_ms",
                                                   "simulate_ms", "finalize_ms", "update_activity_ms")}
        result["large_loop"]["workload"] = ll["config"]["workload"]
        log("[bench] joint-estimation leg")
        result["joint_loop"] = joint_loop(args)
    if not args.no_cpu_baseline:
        log(f"[bench] CPU oracle baseline on {args.cpu_histories} histories")
        result["cpu_baseline"] = cpu_baseline(w, physics, pdesc, mu, act, lut_desc, lut, args.cpu_histories, gaps)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
