"""The allocation-free entry point ddp_loss_and_grad_static (work counters and
activation stash in the library's static device scratch) against
ddp_loss_and_grad on the same handle: two calls in a row, the second on a
smaller problem, and the per-subdomain path; every output bit for bit."""
import sys

import numpy as np
import pytest
import torch

from paper_2104_10013_amd import ddpinn, workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _both(pb):
    lt, g = pb.loss_and_grad()
    torch.cuda.synchronize()
    lt, g = lt.cpu().numpy(), g.cpu().numpy()
    # output buffers first (the caller's allocation), then the call itself
    lt_s = torch.empty(pb.n_sd, 5, dtype=torch.float32, device=pb.device)
    g_s = torch.empty(int(pb.offsets[-1]), dtype=torch.float32, device=pb.device)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    ddpinn._check(ddpinn._lib.ddp_loss_and_grad_static(pb._h, ddpinn._ptr(lt_s), ddpinn._ptr(g_s)))
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    return lt, g, lt_s.cpu().numpy(), g_s.cpu().numpy(), free0, free1


def test_static_scratch_entry_matches_loss_and_grad():
    # first call: the full-size 16-subdomain workload, whose plan wants more
    # stash slots than the static scratch holds (the grid is clamped)
    _say("no-alloc: c2_xpinn_poisson seed 0 full size, fused")
    big = W.c2_xpinn_poisson(seed=0)
    pb = ddpinn.Problem(big, fused=True)
    lt, g, lt_s, g_s, f0, f1 = _both(pb)
    assert np.array_equal(lt, lt_s) and np.array_equal(g, g_s)
    assert np.all(np.isfinite(g)) and np.abs(g).max() > 0
    pb.close()
    # second call, smaller problem: the array keeps the first call's stash and
    # counters; the call zeroes the counters itself and allocates nothing
    _say("no-alloc: c2_xpinn_poisson seed 1 scale 0.05, fused")
    small = W.c2_xpinn_poisson(seed=1, scale=0.05)
    pb = ddpinn.Problem(small, fused=True)
    pb.set_params([W.perturb_params(s.params, 7, 0.1) for s in small.subdomains])
    lt, g, lt_s, g_s, f0, f1 = _both(pb)
    assert np.array_equal(lt, lt_s) and np.array_equal(g, g_s)
    assert f1 == f0, f"device free memory changed across the call: {f0} -> {f1}"
    pb.close()


def test_static_scratch_entry_per_subdomain_path_and_repeat():
    _say("no-alloc: c5_xpinn_inverse_diffusion seed 0 scale 0.05, per-subdomain path, twice")
    prob = W.c5_xpinn_inverse_diffusion(seed=0, scale=0.05)
    pb = ddpinn.Problem(prob, fused=False)
    lt, g, lt_s, g_s, f0, f1 = _both(pb)
    assert np.array_equal(lt, lt_s) and np.array_equal(g, g_s)
    lt2, g2, lt_s2, g_s2, f0, f1 = _both(pb)
    assert np.array_equal(lt_s, lt_s2) and np.array_equal(g_s, g_s2)
    assert f1 == f0
    pb.close()
