"""The joint activity / scatter estimation loop (Methods, "Unknown activity
distribution, very limited simulation time") on the tiny workload: every
step is a library call (OSEM, image to activity, simulation, normalised
smoothing); the loop brings the total scatter estimate close to the true
scatter's and the reconstruction closer to the true image than the
reconstruction without scatter compensation."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2509_05047_amd as sse  # noqa: E402
from paper_2509_05047_amd import joint  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_joint_loop_on_the_tiny_workload():
    w = W.WORKLOADS["tiny"]
    sino = W.Sinogram(**{**w.sino.__dict__, "tof_sigma_mm": 20.0})
    pd, mu, act = W.make_phantom(w)
    ld, lut = W.make_lut(w.lut_dims, w.lut_seed)
    ctx = sse.Context(w.scanner, sino, w.physics)
    try:
        ctx.load_lut(ld, lut)
        ctx.load_sensitivity(W.make_sensitivity(sino, seed=3, tof_axis=True), has_tof_axis=True)
        pid = ctx.load_phantom(pd, mu, act)
        x_true = torch.from_numpy(W.plane_image(pd, act, w.scanner)).cuda()
        detector = torch.from_numpy(W.make_sensitivity(sino, seed=11, tof_axis=False)).cuda()
        prompts, mult, s_true, t = joint.synthetic_acquisition(ctx, pid, x_true, detector, total_prompts=2e7,
                                                               n_histories=50_000_000, noise_seed=None)
        ref_mu, ref_act = W.reference_cylinder(pd, 60.0)
        rid = ctx.load_phantom(pd, ref_mu, ref_act)
        out = ctx.new_outputs()
        ctx.simulate(rid, 20_000_000, 3, out)
        norm = torch.empty(ctx.n_bins, dtype=torch.float32, device="cuda")
        ctx.smoothing_normalisation(out["scatter_weights"], ctx.emission_scale(rid, 20_000_000), norm,
                                    (3.0, 3.0, 1.0))
        del out
        errs = []

        def cb(k, image, scatter):
            errs.append((float((scatter.double().sum() / s_true.double().sum() - 1).abs()),
                         float((image - x_true).norm() / x_true.norm())))

        # the reconstruction without scatter compensation, for comparison
        x_nosc = torch.full_like(x_true, float(x_true.mean()))
        ctx.osem(pid, prompts, mult, torch.zeros_like(prompts), x_nosc, n_iter=4, n_subsets=4)
        torch.cuda.synchronize()
        err_nosc = float((x_nosc - x_true).norm() / x_true.norm())
        image, scatter, timing = joint.joint_estimation(
            ctx, pid, prompts, mult, norm.view(prompts.shape), (1.0, 1.0, 0.5), n_iter=4, n_subsets=4,
            n_histories=4_000_000, seed=41, acq_seconds=t, initial_iterations=1,
            image=torch.full_like(x_true, float(x_true.mean())), callback=cb)
        say(f"[joint] no scatter compensation: image error {err_nosc:.4f}")
        for k, (es, ei) in enumerate(errs):
            say(f"[joint] iteration {k}: total scatter error {es:.4f}, image error {ei:.4f}, "
                f"{timing.iteration_ms[k]:.1f} ms")
        assert len(timing.iteration_ms) == 4
        assert errs[-1][0] < 0.1, errs
        assert errs[-1][1] < err_nosc, (errs, err_nosc)
        assert np.isfinite(image.cpu().numpy()).all()
    finally:
        ctx.close()
