"""Joint activity / scatter estimation loop (Methods, "Unknown activity
distribution, very limited simulation time"): reconstruct the activity with
the current scatter estimate, run a short scatter simulation with that
activity and the known attenuation map, reduce its noise by the normalised
smoothing, and repeat.  The paper runs 10 such iterations with 1 TOF-OSEM
iteration of 28 subsets each, from an initial reconstruction without scatter
compensation.

Every step is a call of the C library (sse_osem with the subset
sensitivity images of sse_osem_sensitivity, sse_image_to_activity,
sse_simulate, sse_finalize_normalised); this module only sequences the calls
and holds the device buffers.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

from . import Context


@dataclass
class LoopTiming:
    """Milliseconds of each loop iteration and of its steps (host clock,
    device synchronised after each step)."""
    iteration_ms: list = field(default_factory=list)
    activity_ms: list = field(default_factory=list)
    simulate_ms: list = field(default_factory=list)
    smooth_ms: list = field(default_factory=list)
    osem_ms: list = field(default_factory=list)
    initial_ms: float = 0.0


def joint_estimation(ctx: Context, pid: int, prompts, mult, norm, sigma_bins, n_iter: int = 10,
                     n_subsets: int = 28, n_histories: int = 1_500_000_000, seed: int = 1,
                     acq_seconds: float = 1.0, factor: float = 1.0, initial_iterations: int = 1,
                     image=None, callback=None, stream=None):
    """Run the loop on phantom `pid` (its attenuation map is the known one; its
    grid is the image grid).  prompts: TOF sinogram; mult: multiplicative
    sinogram without TOF axis (attenuation factors times detector
    sensitivity); norm: smoothing normalisation sinogram; sigma_bins: the
    smoothing's (radial, view, plane) sigmas.  The loaded scatter-sensitivity
    sinogram turns the LUT scatter into the estimate.  Iteration k simulates
    histories [k n, (k + 1) n) of `seed`.  callback(k, image, scatter) after
    each iteration.  Returns (image, scatter estimate, LoopTiming)."""
    import torch
    dev = prompts.device
    pd_ny, pd_nx = ctx.phantom_grid(pid)
    n_plane = ctx.sino.n_plane
    if image is None:
        image = torch.ones((n_plane, pd_ny, pd_nx), dtype=torch.float32, device=dev)
    scatter = torch.zeros_like(prompts)
    out = ctx.new_outputs(trues=False, stats=False)
    timing = LoopTiming()   # initial_ms includes the subset sensitivity images

    def sync():
        torch.cuda.synchronize(dev)
        return time.perf_counter()

    t0 = sync()
    sens = ctx.osem_sensitivity(pid, mult, n_subsets, stream=stream)   # m is the same in every iteration
    ctx.osem(pid, prompts, mult, scatter, image, n_iter=initial_iterations, n_subsets=n_subsets, sens=sens,
             stream=stream)
    timing.initial_ms = (sync() - t0) * 1e3
    for k in range(n_iter):
        t0 = sync()
        ctx.image_to_activity(pid, image, stream=stream)
        t1 = sync()
        out["scatter_counts"].zero_()
        out["scatter_weights"].zero_()
        ctx.simulate(pid, n_histories, seed, out, h_offset=k * n_histories, stream=stream)
        t2 = sync()
        scale = ctx.emission_scale(pid, n_histories, acq_seconds, factor)
        ctx.finalize_normalised(out["scatter_weights"], scale, norm, scatter, sigma_bins, stream=stream)
        t3 = sync()
        ctx.osem(pid, prompts, mult, scatter, image, n_iter=1, n_subsets=n_subsets, sens=sens, stream=stream)
        t4 = sync()
        timing.iteration_ms.append((t4 - t0) * 1e3)
        timing.activity_ms.append((t1 - t0) * 1e3)
        timing.simulate_ms.append((t2 - t1) * 1e3)
        timing.smooth_ms.append((t3 - t2) * 1e3)
        timing.osem_ms.append((t4 - t3) * 1e3)
        if callback is not None:
            callback(k, image, scatter)
    return image, scatter, timing


def synthetic_acquisition(ctx: Context, pid: int, image_true, detector, scatter_fraction: float = 0.34,
                          total_prompts: float = 5e8, n_histories: int = 20_000_000_000, seed: int = 97,
                          noise_seed: int | None = 5, stream=None):
    """A synthetic acquisition for the loop, made with the library's own
    models: trues = kappa * detector * attenuation * (TOF projection of
    image_true) and scatter = a long simulation of phantom pid (which must hold
    the true activity) times the loaded scatter sensitivity; kappa sets the
    scatter fraction, one common time scale t the total counts, and the
    prompts are Poisson draws of their sum (noise_seed None: the expectation).
    detector: detector sensitivity without TOF axis.  Returns (prompts,
    mult = t kappa detector attenuation, true scatter (scaled by t), t) --
    the loop then takes acq_seconds = t."""
    import torch
    dev = image_true.device
    sn = ctx.sino
    att = torch.empty((sn.n_plane, sn.n_view, sn.n_rad), dtype=torch.float32, device=dev)
    ctx.attenuation_factors(pid, att, stream=stream)
    out = ctx.new_outputs(trues=False, stats=False)
    ctx.simulate(pid, n_histories, seed, out, stream=stream)
    scatter = torch.empty((sn.n_tof, sn.n_plane, sn.n_view, sn.n_rad), dtype=torch.float32, device=dev)
    ctx.apply_sensitivity(out["scatter_weights"], ctx.emission_scale(pid, n_histories), scatter, stream=stream)
    del out
    trues = torch.empty_like(scatter)
    ctx.project(pid, image_true, trues, tof=True, stream=stream)
    torch.cuda.synchronize(dev)
    base = detector * att
    trues *= base[None]
    s_sum, t_sum = float(scatter.double().sum()), float(trues.double().sum())
    kappa = s_sum * (1.0 - scatter_fraction) / scatter_fraction / t_sum
    t = total_prompts / (s_sum + kappa * t_sum)
    expected = trues.mul_(kappa * t).add_(scatter, alpha=t)
    if noise_seed is None:
        prompts = expected
    else:
        g = torch.Generator(device=dev).manual_seed(int(noise_seed))
        prompts = torch.poisson(expected, generator=g)
        del expected
    mult = (base * (kappa * t)).contiguous()
    return prompts, mult, scatter.mul_(t), t
