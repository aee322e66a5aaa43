"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle on the
same seeded inputs and float32 parameters."""
import ctypes
import sys

import numpy as np
import pytest
import torch

import oracle
from paper_2104_10013_amd import ddpinn, workloads as W
from parity_util import compare

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run(prob, params=None, fused=True, **kw):
    pb = ddpinn.Problem(prob, fused=fused, **kw)
    if params is not None:
        pb.set_params(params)
    lt, g = pb.loss_and_grad()
    torch.cuda.synchronize()
    return pb, lt.cpu().numpy(), [x.cpu().numpy() for x in pb.split(g.cpu())]


def _params(prob, seed):
    if seed is None:
        return [s.params for s in prob.subdomains]
    return [W.perturb_params(s.params, seed, 0.1) for s in prob.subdomains]


@pytest.mark.parametrize("seed", [None, 11, 12, 13])
def test_c1_cpinn_poisson_full(seed):
    prob = W.c1_cpinn_poisson(seed=0)
    params = _params(prob, seed)
    _say(f"c1 full, perturbation {seed}")
    pb, lt, g = run(prob, params)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    pb.close()


@pytest.mark.parametrize("seed", [None, 21])
def test_c2_xpinn_poisson_scaled(seed):
    prob = W.c2_xpinn_poisson(seed=1, scale=0.1)
    params = _params(prob, seed)
    _say(f"c2 scale 0.1, perturbation {seed}")
    pb, lt, g = run(prob, params)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    pb.close()


def test_c2_xpinn_poisson_full_size_bench_launch():
    """Full-size 16-subdomain workload in the launch configuration the
    benchmark times (fused, work plan chosen by the autotuner), and with the
    default plan."""
    prob = W.c2_xpinn_poisson(seed=0)
    params = _params(prob, None)
    terms, grads = oracle.loss_and_grad(prob, params)
    for tuned in (True, False):
        _say(f"c2 full size, autotuned plan {tuned}")
        pb = ddpinn.Problem(prob, fused=True)
        if tuned:
            _say(f"  plan {pb.autotune(iters=3)}")
        lt, g = pb.loss_and_grad()
        torch.cuda.synchronize()
        wl, wg = compare(prob, params, lt.cpu().numpy(), [x.cpu().numpy() for x in pb.split(g.cpu())],
                         ref=(terms, grads))
        _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
        pb.close()


def test_ragged_mixed_widths_and_depths():
    """Widths across every class (incl. non-multiples of 16), depth 1..6,
    point counts that are not tile multiples, one subdomain without residual
    points, interface counts of 1 and 67."""
    widths = [[2, 20, 1], [2, 33, 33, 1], [2, 50, 50, 50, 50, 1], [2, 80] + [80] * 5 + [1]]
    prob = W.custom_box_problem("xpinn", "poisson2d", 2, 2, widths, [1, 65, 130, 0], n_bnd_seg=3, n_iface=67,
                                seed=3)
    prob.interfaces[0].xy = prob.interfaces[0].xy[:1].copy()
    params = _params(prob, 5)
    _say("ragged mixed widths")
    pb, lt, g = run(prob, params, chunk_points=64)
    compare(prob, params, lt, g)
    pb.close()


@pytest.mark.parametrize("method", ["cpinn", "xpinn"])
def test_two_subdomain_methods(method):
    prob = W.custom_box_problem(method, "poisson2d", 2, 1, [[2, 48, 48, 48, 1], [2, 24, 24, 1]], [300, 257],
                                n_bnd_seg=40, n_iface=129, seed=7)
    params = _params(prob, 8)
    _say(f"two subdomains {method}")
    pb, lt, g = run(prob, params)
    compare(prob, params, lt, g)
    pb.close()


def test_c3_cpinn_burgers_scaled():
    prob = W.c3_cpinn_burgers(seed=0, scale=0.2)
    params = _params(prob, 31)
    _say("c3 burgers scale 0.2")
    pb, lt, g = run(prob, params)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    pb.close()


def test_c4_xpinn_kovasznay_scaled():
    prob = W.c4_xpinn_kovasznay(seed=0, scale=0.1)
    params = _params(prob, 41)
    _say("c4 kovasznay scale 0.1")
    pb, lt, g = run(prob, params)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    pb.close()


def test_fused_matches_plain_and_is_deterministic():
    prob = W.c2_xpinn_poisson(seed=2, scale=0.1)
    _say("fused vs plain")
    pf, lt_f, g_f = run(prob, fused=True)
    lt2, g2 = pf.loss_and_grad()
    torch.cuda.synchronize()
    assert np.array_equal(lt_f, lt2.cpu().numpy())
    assert np.array_equal(np.concatenate(g_f), g2.cpu().numpy())
    pp, lt_p, g_p = run(prob, fused=False)
    np.testing.assert_allclose(lt_p, lt_f, rtol=2e-6, atol=0)
    for a, b in zip(g_p, g_f):
        assert np.linalg.norm(a - b) <= 2e-6 * np.linalg.norm(b)
    pf.close()
    pp.close()


@pytest.mark.parametrize("fused", [True, False])
def test_adam_step_matches_formula(fused):
    prob = W.c1_cpinn_poisson(seed=0, scale=0.3)
    _say(f"adam fused={fused}")
    pb = ddpinn.Problem(prob, fused=fused)
    p0 = pb.get_params()
    _, g = pb.loss_and_grad()
    g = g.cpu().numpy().astype(np.float64)
    lt = pb.step(1)
    st = pb.get_state()
    assert st["t"] == 1
    # (1 - beta) are formed in float32 by the kernel: 1 - 0.999f = 0.00099998713...
    one_m_b1 = float(np.float32(1) - np.float32(0.9))
    one_m_b2 = float(np.float32(1) - np.float32(0.999))
    np.testing.assert_allclose(st["m"], one_m_b1 * g, rtol=1e-6, atol=1e-30)
    np.testing.assert_allclose(st["v"], one_m_b2 * g * g, rtol=1e-6, atol=1e-30)
    for q in range(prob.n_sd):
        gq = pb.split(g)[q]
        ref = p0[q].astype(np.float64) - prob.subdomains[q].lr * gq / (np.abs(gq) + 1e-8)
        np.testing.assert_allclose(st["params"][q], ref, rtol=1e-6, atol=1e-6 * prob.subdomains[q].lr)
    pb.close()


def test_training_trajectory_loosely_follows_oracle():
    """100 Adam steps of the 4-subdomain cPINN Poisson problem at full size:
    every subdomain's loss follows the FP64 oracle's trajectory."""
    prob = W.c1_cpinn_poisson(seed=0)
    n = 100
    _say("trajectory 100 steps")
    pb = ddpinn.Problem(prob, fused=True)
    hist = []
    for _ in range(n):
        hist.append(pb.step(1).cpu().numpy().copy())
    ps_ref, hist_ref = oracle.train(prob, [s.params for s in prob.subdomains], n)
    hist = np.stack(hist)
    np.testing.assert_allclose(hist[:, :, 0], hist_ref[:, :, 0], rtol=1e-3)
    pb.close()


def test_checkpoint_resume_bitwise():
    """50 steps, save, restore into a new problem, 50 more: the same bits as
    100 straight steps."""
    prob = W.c1_cpinn_poisson(seed=0, scale=0.2)
    _say("checkpoint resume")
    a = ddpinn.Problem(prob, fused=True)
    a.step(50)
    st = a.get_state()
    a.step(50)
    pa = a.get_params()
    b = ddpinn.Problem(prob, fused=True)
    b.set_state(st)
    b.step(50)
    pb_ = b.get_params()
    for x, y in zip(pa, pb_):
        assert np.array_equal(x, y)
    assert b.get_state()["t"] == 100
    a.close()
    b.close()


def test_stitched_eval_matches_oracle():
    prob = W.c2_xpinn_poisson(seed=0, scale=0.05)
    _say("stitched eval")
    pb = ddpinn.Problem(prob, fused=True)
    idx = np.arange(0, prob.eval_xy.shape[0], 37)
    u = pb.eval(prob.eval_xy[idx], prob.eval_owner[idx]).cpu().numpy()
    ref = oracle.eval_stitched(prob, [s.params for s in prob.subdomains], prob.eval_xy[idx], prob.eval_owner[idx])
    np.testing.assert_allclose(u, ref, rtol=1e-5, atol=1e-6)
    pb.close()


def test_nonfinite_loss_is_reported():
    prob = W.c1_cpinn_poisson(seed=0, scale=0.1)
    _say("non-finite flag")
    pb = ddpinn.Problem(prob, fused=True)
    pb.sync()
    bad = [s.params.copy() for s in prob.subdomains]
    bad[2][:] = np.nan
    pb.set_params(bad)
    pb.loss_and_grad()
    with pytest.raises(ddpinn.DDPError) as ei:
        pb.sync()
    assert ei.value.code == ddpinn.DDP_ENONFINITE
    pb.set_params([s.params for s in prob.subdomains])
    pb.loss_and_grad()
    pb.sync()
    pb.close()


def test_autograd_function_backward():
    prob = W.c1_cpinn_poisson(seed=0, scale=0.1)
    _say("autograd function")
    pb = ddpinn.Problem(prob, fused=True)
    flat = torch.tensor(np.concatenate([s.params for s in prob.subdomains]), device="cuda", requires_grad=True)
    J = ddpinn.DDPLoss.apply(flat, pb)
    w = torch.tensor([1.0, 2.0, 0.5, -1.0], device="cuda")
    (J * w).sum().backward()
    _, g = pb.loss_and_grad()
    ref = torch.cat([g[pb.offsets[q]:pb.offsets[q + 1]] * w[q] for q in range(4)])
    assert torch.equal(flat.grad, ref)
    pb.close()


@pytest.mark.parametrize("name", ["c3_cpinn_burgers", "c4_xpinn_kovasznay", "c1_cpinn_poisson"])
def test_full_size_configs_at_init(name):
    """Every workload at its full size, fused launch, initial parameters."""
    prob = W.make_problem(name, seed=0)
    params = _params(prob, None)
    _say(f"{name} full size")
    pb, lt, g = run(prob, params)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    pb.close()


def test_c4_adjoint_vs_central_fd_of_oracle_loss():
    """The GPU gradient of a Navier-Stokes subdomain loss against central
    differences (h = 1e-3, FP64) of the oracle's J_q on sampled parameters."""
    prob = W.c4_xpinn_kovasznay(seed=0, scale=0.02)
    params = _params(prob, 5)
    _say("c4 adjoint vs central FD")
    pb, lt, g = run(prob, params)
    rng = np.random.default_rng(0)
    for q in (0, 4):
        idx = rng.choice(len(params[q]), 12, replace=False)
        base = [torch.tensor(p, dtype=torch.float64) for p in params]
        for i in idx:
            h = 1e-3
            bp = [b.clone() for b in base]
            bm = [b.clone() for b in base]
            bp[q][i] += h
            bm[q][i] -= h
            jp = float(oracle.subdomain_terms(prob, q, bp)[0].detach())
            jm = float(oracle.subdomain_terms(prob, q, bm)[0].detach())
            fd = (jp - jm) / (2 * h)
            scale = np.linalg.norm(g[q]) / np.sqrt(len(g[q]))
            assert abs(g[q][i] - fd) <= 1e-3 * max(abs(fd), scale), (q, i, g[q][i], fd)
    pb.close()


def test_autotune_keeps_results_and_caches(tmp_path):
    prob = W.c2_xpinn_poisson(seed=3, scale=0.1)
    _say("autotune")
    pb, lt0, g0 = run(prob)
    cache = tmp_path / "tune.jsonl"
    choice = pb.autotune(iters=2, cache_path=cache)
    assert choice["recompute"] in (0, 1) and choice["concurrent"] in (0, 1) and choice["tail"] in (0, 30)
    assert cache.exists() and len(cache.read_text().splitlines()) == 1
    lt1, g1 = pb.loss_and_grad()
    torch.cuda.synchronize()
    compare(prob, [s.params for s in prob.subdomains], lt1.cpu().numpy(), [x.cpu().numpy() for x in pb.split(g1.cpu())])
    # a second problem with the same signature takes the cached choice without a search
    pb2 = ddpinn.Problem(prob, fused=True)
    assert pb2.autotune(iters=2, cache_path=cache) == choice
    assert len(cache.read_text().splitlines()) == 1
    pb.step(2)
    pb.sync()
    pb.close()
    pb2.close()


# --------------------------------------------------------------------------
# inverse diffusion (Eq. heq): u- and K-network per subdomain, paired items


@pytest.mark.parametrize("seed", [None, 51])
def test_c5_inverse_scaled(seed):
    prob = W.c5_xpinn_inverse_diffusion(seed=0, scale=0.03)
    params = _params(prob, seed)
    _say(f"c5 scale 0.03, perturbation {seed}")
    pb, lt, g = run(prob, params)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    pb.close()


def test_c5_inverse_full_size_bench_launch():
    prob = W.c5_xpinn_inverse_diffusion(seed=0)
    params = _params(prob, None)
    _say("c5 full size")
    pb, lt, g = run(prob, params)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    pb.close()


def test_concurrent_launches_match_sequential_bitwise():
    """Items that need the two train kernels (networks up to 80 and wider):
    the two persistent launches side by side on two streams give the same
    bits as one after the other, in a loss-and-gradient pass and over graph
    steps with Adam; full size against the oracle."""
    prob = W.c5_xpinn_inverse_diffusion(seed=0, scale=0.05)
    params = _params(prob, 7)
    out = {}
    for conc in (0, 1):
        _say(f"c5 scale 0.05 concurrent {conc}")
        pb, lt, g = run(prob, params, concurrent=conc)
        pb.step(3)
        pb.sync()
        out[conc] = (lt, g, pb.get_params())
        pb.close()
    assert np.array_equal(out[0][0], out[1][0])
    for a, b in zip(out[0][1], out[1][1]):
        assert np.array_equal(a, b)
    for a, b in zip(out[0][2], out[1][2]):
        assert np.array_equal(np.asarray(a), np.asarray(b))
    compare(prob, params, out[1][0], out[1][1])
    prob = W.c5_xpinn_inverse_diffusion(seed=0)
    params = _params(prob, None)
    _say("c5 full size concurrent 1")
    pb, lt, g = run(prob, params, concurrent=1)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    pb.close()


def test_c5_inverse_narrow_ragged_fused_and_plain():
    """Narrow and mixed widths for both networks (non-multiples of 16), short
    point sets that end inside a tile, fused and per-subdomain launches."""
    prob = W.c5_xpinn_inverse_diffusion(seed=3, scale=0.01)
    rng = np.random.default_rng(0)
    choices = [[2, 20, 1], [2, 33, 33, 1], [2, 40, 40, 40, 1], [2, 17, 17, 17, 17, 1]]
    for q, s in enumerate(prob.subdomains):
        s.widths = list(choices[q % 4])
        s.aux_widths = list(choices[(q + 1) % 4])
        s.params = np.concatenate([W.glorot_params(rng, s.widths), W.glorot_params(rng, s.aux_widths)])
    params = _params(prob, 7)
    for fused in (True, False):
        _say(f"c5 narrow ragged fused={fused}")
        pb, lt, g = run(prob, params, fused=fused, chunk_points=64)
        compare(prob, params, lt, g)
        pb.close()


def test_c5_stitched_eval_and_adam_step():
    prob = W.c5_xpinn_inverse_diffusion(seed=0, scale=0.02)
    params = _params(prob, 61)
    _say("c5 eval and one Adam step")
    pb = ddpinn.Problem(prob, fused=True)
    pb.set_params(params)
    idx = np.arange(0, prob.eval_xy.shape[0], 23)
    uk = pb.eval(prob.eval_xy[idx], prob.eval_owner[idx]).cpu().numpy()
    ref = oracle.eval_stitched(prob, params, prob.eval_xy[idx], prob.eval_owner[idx])
    assert uk.shape == ref.shape == (idx.size, 2)
    np.testing.assert_allclose(uk, ref, rtol=1e-5, atol=1e-6)
    _, grads = oracle.loss_and_grad(prob, params)
    pb.step(1)
    got = pb.get_params()
    for q, s in enumerate(prob.subdomains):
        th, _, _ = oracle.adam_step(params[q].astype(np.float64), 0.0, 0.0, grads[q], 1, s.lr)
        # step 1 moves every parameter by about lr * sign(g): compare the step
        step = got[q].astype(np.float64) - params[q].astype(np.float64)
        ref_step = th - params[q].astype(np.float64)
        big = np.abs(grads[q]) > 1e-3 * np.abs(grads[q]).max()
        np.testing.assert_allclose(step[big], ref_step[big], rtol=2e-3, atol=2e-6 * s.lr)
    pb.close()


def test_extreme_network_sizes_and_an_empty_subdomain():
    """Maximum sizes (width 112 with 8 hidden layers, the widest class and
    deepest stash), the narrowest networks (widths 1, 3 and 16), Navier-Stokes
    outputs on a wide net, and a subdomain without any points (zero loss and
    gradient, parameters unchanged by Adam)."""
    widths = [[2] + [112] * 8 + [1], [2, 1, 1], [2, 3, 3, 3, 1], [2] + [16] * 7 + [1]]
    prob = W.custom_box_problem("xpinn", "poisson2d", 2, 2, widths, [150, 70, 1, 0], n_bnd_seg=5, n_iface=19,
                                seed=11)
    # the fourth box keeps no points at all: no data, no interfaces
    s3 = prob.subdomains[3]
    s3.bnd_xy, s3.bnd_g = s3.bnd_xy[:0], s3.bnd_g[:0]
    prob.interfaces = [e for e in prob.interfaces if 3 not in (e.a, e.b)]
    params = _params(prob, 13)
    _say("extreme sizes and an empty subdomain")
    pb, lt, g = run(prob, params, chunk_points=64)
    compare(prob, params, lt, g)
    assert np.all(lt[3] == 0) and np.all(g[3] == 0)
    pb.step(1)
    assert np.array_equal(pb.get_params()[3], params[3])
    pb.close()
    prob = W.custom_box_problem("xpinn", "ns2d_steady", 2, 1, [[2] + [112] * 3 + [3], [2, 7, 7, 3]], [90, 40],
                                n_bnd_seg=6, n_iface=23, seed=12, coef=(40.0,), domain=(-0.5, 1.0, -0.5, 1.5))
    params = _params(prob, 14)
    _say("navier-stokes width 112")
    pb, lt, g = run(prob, params)
    compare(prob, params, lt, g)
    pb.close()


def test_c5_training_trajectory_loosely_follows_oracle():
    """30 Adam steps of a small inverse problem (both networks per cell): the
    per-subdomain losses follow the FP64 oracle's trajectory."""
    prob = W.c5_xpinn_inverse_diffusion(seed=1, scale=0.02)
    n = 30
    _say("c5 trajectory 30 steps")
    pb = ddpinn.Problem(prob, fused=True)
    hist = np.stack([pb.step(1).cpu().numpy().copy() for _ in range(n)])
    _, hist_ref = oracle.train(prob, [s.params for s in prob.subdomains], n)
    np.testing.assert_allclose(hist[:, :, 0], hist_ref[:, :, 0], rtol=2e-3)
    pb.close()


@pytest.mark.parametrize("method,nx,nt", W.TABLE3_PARTITIONS)
def test_space_time_burgers_partitions_full_size(method, nx, nt):
    """Every space-time partition of the viscous Burgers comparison (80k
    residual points, 2-20x5-1 networks), at init and perturbed; the 4 x 4
    XPINN and 16-strip cPINN cases also in the autotuned plan and the plain
    path."""
    prob = W.make_problem(f"burgers_st_{method}_{nx}x{nt}", seed=0)
    variants = [(None, True, False)]
    if (method, nx, nt) in (("xpinn", 4, 4), ("cpinn", 16, 1)):
        variants += [(61, True, True), (61, False, False)]
    for seed, fused, tuned in variants:
        params = _params(prob, seed)
        _say(f"burgers {method} {nx}x{nt} perturbation {seed} fused {fused} autotuned {tuned}")
        pb = ddpinn.Problem(prob, fused=fused)
        pb.set_params(params)
        if tuned:
            _say(f"  plan {pb.autotune(iters=3)}")
        lt, g = pb.loss_and_grad()
        torch.cuda.synchronize()
        wl, wg = compare(prob, params, lt.cpu().numpy(), [x.cpu().numpy() for x in pb.split(g.cpu())])
        _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
        pb.close()


def test_space_time_burgers_training_trajectory_loosely_follows_oracle():
    """20 Adam steps of the 2 x 2 space-time XPINN case at a fifth of its
    points: the per-subdomain losses follow the FP64 oracle's trajectory."""
    prob = W.burgers_space_time("xpinn", 2, 2, seed=2, scale=0.2)
    n = 20
    _say("burgers space-time trajectory 20 steps")
    pb = ddpinn.Problem(prob, fused=True)
    hist = np.stack([pb.step(1).cpu().numpy().copy() for _ in range(n)])
    _, hist_ref = oracle.train(prob, [s.params for s in prob.subdomains], n)
    np.testing.assert_allclose(hist[:, :, 0], hist_ref[:, :, 0], rtol=1e-3)
    pb.close()


@pytest.mark.parametrize("scale,seed", [(0.1, 71), (1.0, None)])
def test_ns_cpinn_kovasznay(scale, seed):
    """Navier-Stokes with cPINN interfaces: the momentum and mass fluxes of
    Table 1 matched across the 12 interfaces of the 3 x 3 Kovasznay problem."""
    prob = W.ns_cpinn_kovasznay(seed=0, scale=scale)
    params = _params(prob, seed)
    for fused in ((True, False) if scale < 1 else (True,)):
        _say(f"ns cpinn scale {scale} perturbation {seed} fused {fused}")
        pb, lt, g = run(prob, params, fused=fused)
        wl, wg = compare(prob, params, lt, g)
        _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
        pb.close()


def test_ns_cpinn_ragged_mixed_widths():
    """cPINN Navier-Stokes on 2 x 2 boxes of widths 17..96 with tile-ragged
    point counts and 1..67 interface points."""
    widths = [[2, 17, 17, 3], [2, 40, 40, 40, 3], [2, 64] * 1 + [64] * 3 + [3], [2, 96, 96, 3]]
    prob = W.custom_box_problem("cpinn", "ns2d_steady", 2, 2, widths, [65, 130, 1, 77], n_bnd_seg=5,
                                n_iface=67, seed=9, coef=(40.0,), domain=(-0.5, 1.0, -0.5, 1.5))
    prob.interfaces[1].xy = prob.interfaces[1].xy[:1].copy()
    params = _params(prob, 10)
    _say("ns cpinn ragged mixed widths")
    pb, lt, g = run(prob, params, chunk_points=64)
    compare(prob, params, lt, g)
    pb.close()


@pytest.mark.parametrize("seed", [None, 81])
def test_space_time_burgers_hybrid(seed):
    """cPINN flux matching across the space interfaces and XPINN residual
    continuity across the time interfaces of the 4 x 4 space-time Burgers
    decomposition, in one launch."""
    prob = W.make_problem("burgers_st_hybrid_4x4", seed=0)
    assert {e.method for e in prob.interfaces} == {"cpinn", "xpinn"}
    params = _params(prob, seed)
    _say(f"burgers hybrid 4x4 perturbation {seed}")
    pb, lt, g = run(prob, params)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    pb.close()


# ---------------------------------------------------------------------------
# activation choice and trainable slopes (Sec. 3, Table 4)


def _slope_identity_gaps(sd, theta, grad):
    """a^k dJ/da^k - (<W^k, dJ/dW^k> + <b^k, dJ/db^k>) relative to the terms'
    size, for every hidden layer of each of the subdomain's networks."""
    gaps, off = [], 0
    th, g = theta.astype(np.float64), grad.astype(np.float64)
    for wd in [sd.widths] + ([sd.aux_widths] if sd.aux_widths is not None else []):
        lay = []
        for k in range(1, len(wd)):
            n = wd[k] * wd[k - 1] + wd[k]
            lay.append(slice(off, off + n))
            off += n
        for k in range(len(wd) - 2):
            lhs = th[off + k] * g[off + k]
            prod = th[lay[k]] * g[lay[k]]
            gaps.append(abs(lhs - prod.sum()) / max(np.abs(prod).sum(), 1e-30))
        off += len(wd) - 2
    return gaps


@pytest.mark.parametrize("scale,seed", [(0.05, 91), (1.0, None)])
def test_table4_adaptive_inverse(scale, seed):
    """The inverse problem with Table 4's networks (adaptive tanh / sin / cos
    per subdomain, 3 x 80 for u and K): loss terms and gradients, slopes
    included, against the oracle; at full size also the slope identity of
    every layer on the GPU's own gradient."""
    prob = W.c5_table4_adaptive(seed=0, scale=scale)
    params = _params(prob, seed)
    _say(f"table 4 adaptive scale {scale} perturbation {seed}")
    pb, lt, g = run(prob, params)
    wl, wg = compare(prob, params, lt, g)
    _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
    if scale == 1.0:
        worst = max(max(_slope_identity_gaps(s, params[q], g[q])) for q, s in enumerate(prob.subdomains))
        _say(f"  slope identity worst {worst:.2e}")
        assert worst < 1e-4
    pb.close()


def _mixed_activation_problem(method, pde):
    """2 x 2 boxes across width classes: a plain tanh network, then adaptive
    sin, cos and tanh networks (neighbours of different kinds)."""
    if pde == "poisson2d":
        widths = [[2, 20, 20, 1], [2, 40, 40, 40, 1], [2, 64, 64, 1], [2, 96, 96, 96, 1]]
        prob = W.custom_box_problem(method, pde, 2, 2, widths, [65, 130, 1, 200], n_bnd_seg=7, n_iface=67, seed=12)
    else:
        widths = [[2, 17, 17, 3], [2, 48, 48, 3], [2, 33, 33, 33, 3], [2, 80, 80, 3]]
        prob = W.custom_box_problem(method, pde, 2, 2, widths, [70, 64, 129, 90], n_bnd_seg=5, n_iface=41, seed=13,
                                    coef=(40.0,), domain=(-0.5, 1.0, -0.5, 1.5))
    W.with_activations(prob, ("tanh", "sin", "cos", "tanh"))
    s0 = prob.subdomains[0]
    s0.adaptive, s0.params = False, s0.params[:W.param_count(s0.widths)].copy()
    return prob


@pytest.mark.parametrize("method,pde", [("xpinn", "poisson2d"), ("cpinn", "poisson2d"), ("cpinn", "ns2d_steady")])
def test_mixed_activations_across_classes(method, pde):
    prob = _mixed_activation_problem(method, pde)
    params = _params(prob, 14)
    for fused in (True, False):
        _say(f"mixed activations {method} {pde} fused {fused}")
        pb, lt, g = run(prob, params, fused=fused, chunk_points=64)
        wl, wg = compare(prob, params, lt, g)
        _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
        pb.close()


def test_adaptive_sin_burgers_space_time():
    """Adaptive sin and cos networks on the space-time Burgers problem (only
    u_xx in the second-order stream)."""
    prob = W.with_activations(W.burgers_space_time("xpinn", 2, 2, seed=3, scale=0.02), ("sin", "cos"))
    params = _params(prob, 15)
    _say("adaptive burgers space-time")
    pb, lt, g = run(prob, params)
    compare(prob, params, lt, g)
    pb.close()


def test_table4_eval_adam_and_trajectory():
    """Stitched evaluation with the activations and slopes, one Adam step
    (slopes included) and 20 steps of loss history against the oracle."""
    prob = W.c5_table4_adaptive(seed=1, scale=0.02)
    params = _params(prob, 16)
    _say("table 4 eval, Adam step, trajectory")
    pb = ddpinn.Problem(prob, fused=True)
    pb.set_params(params)
    idx = np.arange(0, prob.eval_xy.shape[0], 23)
    uk = pb.eval(prob.eval_xy[idx], prob.eval_owner[idx]).cpu().numpy()
    ref = oracle.eval_stitched(prob, params, prob.eval_xy[idx], prob.eval_owner[idx])
    np.testing.assert_allclose(uk, ref, rtol=1e-5, atol=1e-6)
    _, grads = oracle.loss_and_grad(prob, params)
    pb.step(1)
    got = pb.get_params()
    for q, s in enumerate(prob.subdomains):
        th, _, _ = oracle.adam_step(params[q].astype(np.float64), 0.0, 0.0, grads[q], 1, s.lr)
        step = got[q].astype(np.float64) - params[q].astype(np.float64)
        ref_step = th - params[q].astype(np.float64)
        big = np.abs(grads[q]) > 1e-3 * np.abs(grads[q]).max()
        np.testing.assert_allclose(step[big], ref_step[big], rtol=2e-3, atol=2e-6 * s.lr)
    pb.close()
    pb = ddpinn.Problem(prob, fused=True)
    pb.set_params(params)
    hist = np.stack([pb.step(1).cpu().numpy().copy() for _ in range(20)])
    _, hist_ref = oracle.train(prob, params, 20)
    np.testing.assert_allclose(hist[:, :, 0], hist_ref[:, :, 0], rtol=2e-3)
    pb.close()


def test_mfma_probe_rate():
    """The attainable FP32 MFMA rate: positive, at most the published peak
    (157.3 TFLOP/s, with a margin for timing), and well above what a
    one-wave-per-SIMD latency-bound loop would show."""
    t = ddpinn.mfma_probe(2000)
    _say(f"mfma probe {t:.1f} TFLOP/s")
    assert 60.0 < t < 165.0


def test_cpinn_burgers_time_interfaces():
    """cPINN across space and time interfaces of 2 x 3 space-time boxes: the
    time component u of the space-time flux and its adjoint."""
    prob = W.burgers_space_time("cpinn", 2, 3, seed=4, scale=0.05)
    assert any(tuple(e.normal) == (0.0, 1.0) for e in prob.interfaces)
    params = _params(prob, 17)
    _say("cpinn burgers with time interfaces")
    for fused in (True, False):
        pb, lt, g = run(prob, params, fused=fused)
        compare(prob, params, lt, g)
        pb.close()


def test_general_activation_kernels_match_plain_bitwise():
    """A tanh problem runs in the plain kernels; the same problem with one
    extra, unconnected sin subdomain runs in the general-activation kernels.
    With one tile per work item (the same summation order), the tanh
    subdomains' loss terms and gradients agree bit for bit."""
    base = W.custom_box_problem("xpinn", "poisson2d", 2, 2,
                                [[2, 20, 20, 1], [2, 48, 48, 48, 1], [2, 64, 64, 1], [2, 80, 80, 80, 1]],
                                [130, 257, 64, 199], n_bnd_seg=9, n_iface=77, seed=21)
    extra = W.custom_box_problem("xpinn", "poisson2d", 1, 1, [[2, 33, 33, 1]], [90], n_bnd_seg=5, n_iface=1,
                                 seed=22, domain=(2.0, 3.0, 0.0, 1.0))
    W.with_activations(extra, ("sin",))
    mixed = W.custom_box_problem("xpinn", "poisson2d", 2, 2,
                                 [[2, 20, 20, 1], [2, 48, 48, 48, 1], [2, 64, 64, 1], [2, 80, 80, 80, 1]],
                                 [130, 257, 64, 199], n_bnd_seg=9, n_iface=77, seed=21)
    mixed.subdomains.append(extra.subdomains[0])
    params = _params(base, 23)
    _say("general-activation kernels vs plain, bitwise")
    pa, la, ga = run(base, params, chunk_points=64)
    pb, lb, gb = run(mixed, params + [extra.subdomains[0].params], chunk_points=64)
    assert np.array_equal(la, lb[:4])
    for q in range(4):
        assert np.array_equal(ga[q], gb[q])
    pa.close()
    pb.close()


def test_phase_timing_of_the_fused_step():
    """Train time split by point kind on the 16-subdomain problem: residual
    items dominate, every phase is timed, and the phases add up to at least
    the whole launch (their separate launches cannot overlap)."""
    prob = W.c2_xpinn_poisson(seed=0)
    pb = ddpinn.Problem(prob, fused=True)
    pb.step(2)
    ph = pb.time_phases(5)
    kt = pb.time_kernels(5)
    _say(f"phases {ph} kernels {kt}")
    assert ph["residual_ms"] > ph["interface_ms"] > 0 and ph["data_ms"] > 0
    assert ph["residual_ms"] + ph["interface_ms"] + ph["data_ms"] >= 0.9 * ph["all_ms"]
    assert 0.5 * kt["train_ms"] < ph["all_ms"] < 2.0 * kt["train_ms"]
    pl = ddpinn.Problem(prob, fused=False)
    with pytest.raises(ddpinn.DDPError):
        pl.time_phases(1)
    pl.close()
    pb.close()


def test_many_subdomains_random_widths_and_depths():
    """64 subdomains (8 x 8, XPINN Poisson) with a random width from 16 to 112
    and 1-6 hidden layers each, ragged residual counts (some empty) and 1-90
    points per interface: both width-class launches, both paths."""
    rng = np.random.default_rng(31)
    widths = [[2] + [int(rng.integers(16, 113))] * int(rng.integers(1, 7)) + [1] for _ in range(64)]
    counts = [int(c) if c > 20 else 0 for c in rng.integers(0, 400, 64)]
    prob = W.custom_box_problem("xpinn", "poisson2d", 8, 8, widths, counts, n_bnd_seg=6, n_iface=90, seed=32)
    for e in prob.interfaces:
        e.xy = e.xy[: int(rng.integers(1, 91))].copy()
    params = _params(prob, 33)
    for fused in (True, False):
        _say(f"64 random subdomains fused {fused}")
        pb, lt, g = run(prob, params, fused=fused)
        wl, wg = compare(prob, params, lt, g)
        _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
        pb.close()


@pytest.mark.parametrize("name,scale", [("c2_xpinn_poisson", 0.1), ("c5_xpinn_inverse_diffusion", 0.03),
                                        ("c5_table4_adaptive", 0.1), ("c3_cpinn_burgers", 0.2),
                                        ("burgers_st_xpinn_2x2", 0.2), ("burgers_st_cpinn_4x1", 0.2)])
def test_recompute_policy(name, scale):
    """Both activation policies (stash a^k and h^k; stash a^k and rebuild h^k
    in the reverse pass) against the oracle, on both paths.  The space-time
    Burgers cases (narrow networks: layer 1 is short, so the next layer's
    weights are still in flight to LDS at the barrier that hands them to the
    other waves unless every wave waits for its own copies) run the fused
    path three times."""
    prob = W.make_problem(name, seed=0, scale=scale)
    params = _params(prob, 5)
    ref = oracle.loss_and_grad(prob, params)
    reps = 3 if name.startswith("burgers_st") else 1
    for fused in (True, False):
        for rh in (0, 1):
            for _ in range(reps if fused else 1):
                _say(f"{name} scale {scale} fused {fused} recompute {rh}")
                pb, lt, g = run(prob, params, fused=fused, recompute=rh)
                wl, wg = compare(prob, params, lt, g, ref=ref)
                _say(f"  worst loss rel {wl:.2e} grad rel {wg:.2e}")
                pb.close()


@pytest.mark.parametrize("name,scale,seed", [("c2_xpinn_poisson", 0.1, 1), ("burgers_st_xpinn_2x2", 0.2, 0),
                                             ("c5_xpinn_inverse_diffusion", 0.03, 0)])
def test_work_plans_against_oracle(name, scale, seed):
    """The work plans the autotuner chooses among (points per item, items per
    workgroup, workgroups per CU, activation policy, tail share of one-tile
    items, and for the inverse problem side-by-side launches) all give the
    oracle's loss and gradient."""
    prob = W.make_problem(name, seed=seed, scale=scale)
    params = _params(prob, 3)
    ref = oracle.loss_and_grad(prob, params)
    conc = (0, 1) if name.startswith("c5") else (0,)
    worst = 0.0
    for chunk in (64, 512, 4096):
        for ips in (1, 8):
            for bpc in (1, 2):
                for rh in (0, 1):
                    for cc in conc:
                        tail = 30 if (ips == 8) == (rh == 1) else 0
                        pb, lt, g = run(prob, params, chunk_points=chunk, items_per_slot=ips, blocks_per_cu=bpc,
                                        recompute=rh, concurrent=cc, tail=tail)
                        try:
                            wl, wg = compare(prob, params, lt, g, ref=ref)
                        except AssertionError:
                            _say(f"{name} plan {chunk}/{ips}/{bpc}/rh{rh}/c{cc} failed")
                            raise
                        worst = max(worst, wl, wg)
                        pb.close()
    _say(f"{name}: every plan within the bar, worst {worst:.2e}")
