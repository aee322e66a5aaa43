"""Pins of the FP64 oracle against mathematics it does not itself compute:
finite differences, closed forms, exact solutions, invariants and a library
optimiser.  A dropped term, a wrong sign or index in the oracle fails one of
these."""
import math

import numpy as np
import pytest
import torch

import oracle
from oracle import pinn_oracle as O
from paper_2104_10013_amd import workloads as W

DT = torch.float64


def _rand_theta(rng, widths, scale=1.0):
    p = W.glorot_params(rng, widths).astype(np.float64)
    # non-zero biases so every parameter is exercised
    off = 0
    for k in range(1, len(widths)):
        off += widths[k] * widths[k - 1]
        p[off:off + widths[k]] = rng.normal(0, 0.3, widths[k])
        off += widths[k]
    return torch.tensor(p * scale, dtype=DT)


# --------------------------------------------------------------------------
# input derivatives (Taylor quantities) vs central finite differences


@pytest.mark.parametrize("widths,pde", [([2, 5, 5, 1], "poisson2d"), ([2, 4, 6, 4, 3], "ns2d_steady"),
                                        ([2, 5, 5, 1], "burgers1d")])
def test_input_streams_vs_central_fd(widths, pde):
    rng = np.random.default_rng(1)
    th = _rand_theta(rng, widths)
    z = torch.tensor(rng.uniform(-1, 1, (7, 2)), dtype=DT)
    st = O.input_streams(th, widths, z, pde, create_graph=False)
    f = lambda zz: O.mlp(th, widths, zz).detach()
    h1, h2 = 1e-5, 1e-3
    S = O.second_order_set(pde)
    lap = torch.zeros_like(st["lap"])
    for i in range(2):
        e = torch.zeros(2, dtype=DT)
        e[i] = 1
        dfd = (f(z + h1 * e) - f(z - h1 * e)) / (2 * h1)
        assert torch.allclose(st["du"][:, :, i], dfd, rtol=1e-7, atol=1e-8)
        if i in S:
            lap += (f(z + h2 * e) - 2 * f(z) + f(z - h2 * e)) / (h2 * h2)
    assert torch.allclose(st["lap"], lap, rtol=1e-5, atol=1e-6)


def test_one_neuron_closed_form():
    # u = c tanh(w1 x + w2 y + b) + d
    w1, w2, b, c, d = 0.7, -1.3, 0.2, 1.9, -0.4
    th = torch.tensor([w1, w2, b, c, d], dtype=DT)
    z = torch.tensor([[0.3, 0.1], [-0.5, 0.8], [1.2, -0.7]], dtype=DT)
    st = O.input_streams(th, [2, 1, 1], z, "poisson2d", create_graph=False)
    a = w1 * z[:, 0] + w2 * z[:, 1] + b
    t = torch.tanh(a)
    s1 = 1 / torch.cosh(a) ** 2
    assert torch.allclose(st["u"][:, 0], c * t + d, rtol=1e-14)
    assert torch.allclose(st["du"][:, 0, 0], c * s1 * w1, rtol=1e-13)
    assert torch.allclose(st["du"][:, 0, 1], c * s1 * w2, rtol=1e-13)
    lap = c * (-2 * t * s1) * (w1 ** 2 + w2 ** 2)
    assert torch.allclose(st["lap"][:, 0], lap, rtol=1e-12)


# --------------------------------------------------------------------------
# residual operators: exact solutions give F == 0


def _pts(n=50, seed=3, lo=0.0, hi=1.0):
    return np.random.default_rng(seed).uniform(lo, hi, (n, 2))


def test_poisson_exact_solution_zero_residual():
    p = _pts()
    x, y = p[:, 0], p[:, 1]
    pi = math.pi
    st = {"u": torch.tensor(np.sin(pi * x) * np.sin(pi * y))[:, None],
          "du": torch.tensor(np.stack([pi * np.cos(pi * x) * np.sin(pi * y),
                                       pi * np.sin(pi * x) * np.cos(pi * y)], 1))[:, None, :],
          "lap": torch.tensor(-2 * pi * pi * np.sin(pi * x) * np.sin(pi * y))[:, None]}
    f = torch.tensor(W.poisson_forcing(x, y))[:, None]
    F = O.residual("poisson2d", (), st, f)
    assert F.abs().max() < 1e-12


def test_kovasznay_exact_solution_zero_residual():
    re = 40.0
    lam = W.kovasznay_lambda(re)
    p = _pts(lo=-0.5, hi=1.0)
    x, y = p[:, 0], p[:, 1]
    e = np.exp(lam * x)
    c, s = np.cos(2 * np.pi * y), np.sin(2 * np.pi * y)
    k = 2 * np.pi
    u = 1 - e * c
    v = lam / k * e * s
    pr = 0.5 * (1 - e * e)
    ux, uy = -lam * e * c, k * e * s
    vx, vy = lam * lam / k * e * s, lam * e * c
    px, py = -lam * e * e, 0 * x
    lapu = -(lam * lam - k * k) * e * c
    lapv = lam / k * (lam * lam - k * k) * e * s
    st = {"u": torch.tensor(np.stack([u, v, pr], 1)),
          "du": torch.tensor(np.stack([np.stack([ux, uy], 1), np.stack([vx, vy], 1),
                                       np.stack([px, py], 1)], 1)),
          "lap": torch.tensor(np.stack([lapu, lapv, 0 * x], 1))}
    F = O.residual("ns2d_steady", (re,), st, torch.zeros(len(x), 3, dtype=DT))
    assert F.abs().max() < 1e-12
    # and the closed form of the workload matches these fields
    np.testing.assert_allclose(W.kovasznay_exact(x, y, re), np.stack([u, v, pr], 1), rtol=1e-14)


def test_burgers_travelling_wave_zero_residual():
    # u = c - a tanh(a (x - c t) / (2 nu)) solves u_t + u u_x = nu u_xx
    nu, a, c = 0.05, 0.8, 0.3
    p = _pts(lo=-1, hi=1)
    x, t = p[:, 0], p[:, 1]
    xi = a * (x - c * t) / (2 * nu)
    th, sech2 = np.tanh(xi), 1 / np.cosh(xi) ** 2
    u = c - a * th
    ux = -a * a / (2 * nu) * sech2
    ut = -c * ux
    uxx = a ** 3 / (2 * nu * nu) * th * sech2
    st = {"u": torch.tensor(u)[:, None], "du": torch.tensor(np.stack([ux, ut], 1))[:, None, :],
          "lap": torch.tensor(uxx)[:, None]}
    F = O.residual("burgers1d", (nu,), st, torch.zeros(len(x), 1, dtype=DT))
    assert F.abs().max() < 1e-10


def test_poisson_flux_and_burgers_flux_closed_form():
    st = {"u": torch.tensor([[0.5]], dtype=DT), "du": torch.tensor([[[2.0, -3.0]]], dtype=DT),
          "lap": torch.zeros(1, 1, dtype=DT)}
    n = torch.tensor([0.6, 0.8], dtype=DT)
    assert float(O.normal_flux("poisson2d", (), st, n)) == pytest.approx(-(0.6 * 2 - 0.8 * 3))
    nu = 0.1
    got = float(O.normal_flux("burgers1d", (nu,), st, torch.tensor([1.0, 0.0], dtype=DT)))
    assert got == pytest.approx(0.5 * 0.25 - nu * 2.0)


# --------------------------------------------------------------------------
# loss assembly


def test_zero_network_gives_mean_forcing_squared():
    prob = W.c1_cpinn_poisson(seed=0)
    params = [np.zeros_like(s.params) for s in prob.subdomains]
    terms, grads = O.loss_and_grad(prob, params)
    for q, s in enumerate(prob.subdomains):
        f = s.res_f.astype(np.float64)[:, 0]
        g = s.bnd_g.astype(np.float64)[:, 0]
        assert terms[q, 2] == pytest.approx(np.mean(f * f), rel=1e-13)
        assert terms[q, 1] == pytest.approx(np.mean(g * g), abs=1e-15)
        assert terms[q, 3] == 0 and terms[q, 4] == 0
    # Monte Carlo estimate of E[f^2] = pi^4 over the unit square
    allf = np.concatenate([s.res_f[:, 0] for s in prob.subdomains]).astype(np.float64)
    assert np.mean(allf ** 2) == pytest.approx(math.pi ** 4, rel=0.05)


def _two_box(method="xpinn", seed=0, n_res=40, widths=(2, 6, 6, 1)):
    return W.custom_box_problem(method, "poisson2d", 2, 1, [list(widths)] * 2, [n_res, n_res + 3],
                                n_bnd_seg=9, n_iface=11, seed=seed)


@pytest.mark.parametrize("method", ["cpinn", "xpinn"])
def test_identical_networks_zero_interface_terms(method):
    prob = _two_box(method)
    p = prob.subdomains[0].params
    terms, grads = O.loss_and_grad(prob, [p, p.copy()])
    assert terms[0, 3] == 0 and terms[0, 4] == 0 and terms[1, 3] == 0 and terms[1, 4] == 0
    # the gradient then equals that of the data and residual terms alone
    prob2 = _two_box(method)
    for s in prob2.subdomains:
        s.loss_w = (1.0, 1.0, 0.0, 0.0)
    _, g2 = O.loss_and_grad(prob2, [p, p.copy()])
    for q in range(2):
        np.testing.assert_allclose(grads[q], g2[q], rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("method", ["cpinn", "xpinn"])
def test_interface_terms_symmetric(method):
    prob = _two_box(method)
    terms, _ = O.loss_and_grad(prob, [s.params for s in prob.subdomains])
    assert terms[0, 3] == pytest.approx(terms[1, 3], rel=1e-14)
    assert terms[0, 4] == pytest.approx(terms[1, 4], rel=1e-14)
    assert terms[0, 3] > 0 and terms[0, 4] > 0
    # J is the weighted sum of its terms
    for q in range(2):
        assert terms[q, 0] == pytest.approx(terms[q, 1:].sum(), rel=1e-14)


def test_uavg_term_is_quarter_of_squared_jump():
    # |u_q - (u_q + u_q+)/2|^2 = (u_q - u_q+)^2 / 4, averaged over the N_e points
    prob = _two_box("xpinn")
    params = [s.params for s in prob.subdomains]
    e = prob.interfaces[0]
    ua = O.mlp(torch.tensor(params[0], dtype=DT), prob.subdomains[0].widths, torch.tensor(e.xy, dtype=DT))
    ub = O.mlp(torch.tensor(params[1], dtype=DT), prob.subdomains[1].widths, torch.tensor(e.xy, dtype=DT))
    ref = float(((ua - ub) ** 2).mean()) / 4
    terms, _ = O.loss_and_grad(prob, params)
    assert terms[0, 3] == pytest.approx(ref, rel=1e-13)


# --------------------------------------------------------------------------
# gradient


def _fd_grad(prob, params, q, h=1e-6, idx=None):
    base = [np.asarray(p, np.float64) for p in params]
    n = base[q].size
    idx = range(n) if idx is None else idx
    g = np.zeros(n)
    for i in idx:
        pp = [b.copy() for b in base]
        pm = [b.copy() for b in base]
        pp[q][i] += h
        pm[q][i] -= h
        thp = [torch.tensor(x, dtype=DT) for x in pp]
        thm = [torch.tensor(x, dtype=DT) for x in pm]
        jp = float(O.subdomain_terms(prob, q, thp)[0])
        jm = float(O.subdomain_terms(prob, q, thm)[0])
        g[i] = (jp - jm) / (2 * h)
    return g


@pytest.mark.parametrize("method", ["cpinn", "xpinn"])
def test_gradient_vs_central_fd_poisson(method):
    prob = W.custom_box_problem(method, "poisson2d", 2, 1, [[2, 3, 3, 1], [2, 3, 3, 1]], [13, 9],
                                n_bnd_seg=5, n_iface=7, seed=4)
    params = [W.perturb_params(s.params, 9, 0.3) for s in prob.subdomains]
    _, grads = O.loss_and_grad(prob, params)
    for q in range(2):
        fd = _fd_grad(prob, params, q)
        np.testing.assert_allclose(grads[q], fd, rtol=2e-6, atol=1e-8)


def test_gradient_vs_central_fd_ns_and_burgers():
    prob = W.custom_box_problem("xpinn", "ns2d_steady", 2, 1, [[2, 3, 3, 3], [2, 4, 3]], [8, 6],
                                n_bnd_seg=4, n_iface=5, seed=5, coef=(40.0,), domain=(-0.5, 1.0, -0.5, 1.5))
    params = [W.perturb_params(s.params, 2, 0.3) for s in prob.subdomains]
    _, grads = O.loss_and_grad(prob, params)
    for q in range(2):
        np.testing.assert_allclose(grads[q], _fd_grad(prob, params, q), rtol=2e-6, atol=1e-8)
    prob = W.c3_cpinn_burgers(seed=1, scale=0.004, n_strips=2)
    for s in prob.subdomains:
        s.widths = [2, 3, 3, 1]
        s.params = W.glorot_params(np.random.default_rng(0), s.widths)
    params = [W.perturb_params(s.params, 3, 0.3) for s in prob.subdomains]
    _, grads = O.loss_and_grad(prob, params)
    for q in range(2):
        np.testing.assert_allclose(grads[q], _fd_grad(prob, params, q), rtol=2e-6, atol=1e-8)


@pytest.mark.parametrize("method", ["cpinn", "xpinn"])
def test_local_gradient_vs_gradient_of_total(method):
    """grad_q sum_r J_r = grad_q J_q + (interface part of grad_q J_q) under
    equal weights: separates the paper's per-subdomain reading from grad(sum)."""
    prob = _two_box(method, seed=2)
    params = [W.perturb_params(s.params, 1, 0.2) for s in prob.subdomains]
    _, g_local = O.loss_and_grad(prob, params)
    g_total = O.grad_of_total(prob, params)
    prob_i = _two_box(method, seed=2)
    for s in prob_i.subdomains:
        s.loss_w = (0.0, 0.0, 1.0, 1.0)
    _, g_iface = O.loss_and_grad(prob_i, params)
    for q in range(2):
        np.testing.assert_allclose(g_total[q], g_local[q] + g_iface[q], rtol=1e-10, atol=1e-13)
        assert np.linalg.norm(g_iface[q]) > 1e-6


# --------------------------------------------------------------------------
# Adam


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(0)
    th, g = rng.normal(size=20), rng.normal(size=20)
    lr = 1e-3
    th1, m, v = O.adam_step(th, np.zeros(20), np.zeros(20), g, 1, lr)
    np.testing.assert_allclose(th1, th - lr * g / (np.abs(g) + 1e-8), rtol=1e-15, atol=1e-18)


def test_adam_matches_torch_optim():
    rng = np.random.default_rng(1)
    th = rng.normal(size=30)
    p = torch.tensor(th.copy(), dtype=DT, requires_grad=True)
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    m = np.zeros(30)
    v = np.zeros(30)
    for t in range(1, 8):
        g = rng.normal(size=30)
        p.grad = torch.tensor(g, dtype=DT)
        opt.step()
        th, m, v = O.adam_step(th, m, v, g, t, 3e-3)
    np.testing.assert_allclose(th, p.detach().numpy(), rtol=1e-13, atol=1e-15)


# --------------------------------------------------------------------------
# stitched solution


def test_stitched_eval_averages_on_interfaces():
    prob = W.c1_cpinn_poisson(seed=0, scale=0.05)
    params = [s.params for s in prob.subdomains]
    xy = np.array([[0.25, 0.25], [0.5, 0.25], [0.5, 0.5], [0.75, 0.9]], np.float32)
    owner = np.array([[0, -1, -1, -1], [0, 1, -1, -1], [0, 1, 2, 3], [3, -1, -1, -1]], np.int32)
    u = O.eval_stitched(prob, params, xy, owner)
    ind = [O.mlp(torch.tensor(p, dtype=DT), s.widths, torch.tensor(xy, dtype=DT)).numpy()[:, 0]
           for p, s in zip(params, prob.subdomains)]
    assert u[0, 0] == pytest.approx(ind[0][0])
    assert u[1, 0] == pytest.approx(0.5 * (ind[0][1] + ind[1][1]))
    assert u[2, 0] == pytest.approx(0.25 * sum(ind[k][2] for k in range(4)))
    assert u[3, 0] == pytest.approx(ind[3][3])
    # the workload's owner table marks the centre cross point with all 4 boxes
    i = np.nonzero((np.abs(prob.eval_xy[:, 0] - 0.5) < 1e-7) & (np.abs(prob.eval_xy[:, 1] - 0.5) < 1e-7))[0]
    assert len(i) == 1 and (prob.eval_owner[i[0]] >= 0).sum() == 4


def test_burgers_reference_solution():
    nu = 0.01 / math.pi
    x = np.linspace(-1, 1, 9)
    np.testing.assert_allclose(W.burgers_exact(x, np.zeros_like(x), nu), -np.sin(np.pi * x), atol=1e-15)
    # boundary values stay 0 and quadrature has converged
    t = np.full(3, 0.5)
    xb = np.array([-1.0, 0.37, 1.0])
    u1 = W.burgers_exact(xb, t, nu, n_nodes=120)
    u2 = W.burgers_exact(xb, t, nu, n_nodes=240)
    assert abs(u1[0]) < 1e-10 and abs(u1[2]) < 1e-10
    np.testing.assert_allclose(u1, u2, atol=1e-8)
    # odd symmetry u(-x,t) = -u(x,t)
    np.testing.assert_allclose(W.burgers_exact(-xb, t, nu), -u1, atol=1e-10)


# --------------------------------------------------------------------------
# inverse diffusion problem (Eq. heq): u-network and K-network per subdomain


def _tiny_c5(seed=1, scale=0.01, wu=(2, 3, 3, 1), wk=(2, 4, 4, 1)):
    """The config-5 geometry and point sets with tiny networks (gradient checks)."""
    prob = W.c5_xpinn_inverse_diffusion(seed=seed, scale=scale)
    rng = np.random.default_rng(seed + 100)
    for s in prob.subdomains:
        s.widths, s.aux_widths = list(wu), list(wk)
        s.params = np.concatenate([W.glorot_params(rng, s.widths), W.glorot_params(rng, s.aux_widths)])
    return prob


def test_inverse_operator_vs_divergence_form_fd():
    """K Lap u + grad K . grad u equals div(K grad u) evaluated by nested central
    differences of the two networks (the form Eq. heq is written in)."""
    rng = np.random.default_rng(7)
    wu, wk = [2, 5, 5, 1], [2, 4, 6, 1]
    thu, thk = _rand_theta(rng, wu), _rand_theta(rng, wk)
    z = torch.tensor(rng.uniform(0.2, 0.8, (9, 2)), dtype=DT)
    stu = O.input_streams(thu, wu, z, O.DIFF_INV, create_graph=False)
    stk = O.input_streams(thk, wk, z, O.DIFF_INV, create_graph=False)
    L = O.residual_inverse(stu, stk, torch.zeros((9, 1), dtype=DT))[:, 0]
    U = lambda zz: O.mlp(thu, wu, zz)[:, 0].detach()
    K = lambda zz: O.mlp(thk, wk, zz)[:, 0].detach()
    hi, ho = 1e-5, 1e-3

    def flux(zz, i):   # K du/dz_i by a central difference
        e = torch.zeros(2, dtype=DT)
        e[i] = hi
        return K(zz) * (U(zz + e) - U(zz - e)) / (2 * hi)

    div = torch.zeros(9, dtype=DT)
    for i in range(2):
        e = torch.zeros(2, dtype=DT)
        e[i] = ho
        div += (flux(z + e, i) - flux(z - e, i)) / (2 * ho)
    np.testing.assert_allclose(L.numpy(), div.numpy(), rtol=2e-5, atol=2e-6)


def test_inverse_exact_fields_zero_residual():
    """The paper's fields T = 20 exp(-0.1 y), K = 20 + exp(0.1 y) sin(0.5 x) satisfy
    Eq. heq with f = 4 exp(-0.1 y) (worked out by hand); the generator's
    manufactured pair satisfies it with its own forcing."""
    p = _pts(40, seed=11)
    x, y = torch.tensor(p[:, 0], dtype=DT), torch.tensor(p[:, 1], dtype=DT)
    e = torch.exp(-0.1 * y)
    stu = {"u": (20 * e)[:, None], "du": torch.stack([0 * x, -2 * e], 1)[:, None, :],
           "lap": (0.2 * e)[:, None]}
    Kv = 20 + torch.sin(0.5 * x) / e
    stk = {"u": Kv[:, None], "du": torch.stack([0.5 * torch.cos(0.5 * x) / e, 0.1 * torch.sin(0.5 * x) / e],
                                               1)[:, None, :]}
    F = O.residual_inverse(stu, stk, (4 * e)[:, None])
    assert float(F.abs().max()) < 1e-12
    # generator's pair: u = sin(pi x) sin(pi y), K = 1 + 0.5 sin(2 pi x) cos(2 pi y)
    pi = math.pi
    u = torch.sin(pi * x) * torch.sin(pi * y)
    stu = {"u": u[:, None], "du": torch.stack([pi * torch.cos(pi * x) * torch.sin(pi * y),
                                               pi * torch.sin(pi * x) * torch.cos(pi * y)], 1)[:, None, :],
           "lap": (-2 * pi * pi * u)[:, None]}
    stk = {"u": (1 + 0.5 * torch.sin(2 * pi * x) * torch.cos(2 * pi * y))[:, None],
           "du": torch.stack([pi * torch.cos(2 * pi * x) * torch.cos(2 * pi * y),
                              -pi * torch.sin(2 * pi * x) * torch.sin(2 * pi * y)], 1)[:, None, :]}
    _, _, f = W.diffusion_fields(p[:, 0], p[:, 1])
    F = O.residual_inverse(stu, stk, torch.tensor(f, dtype=DT)[:, None])
    assert float(F.abs().max()) < 1e-11


def test_inverse_zero_networks_closed_forms():
    """u = K = 0: MSE_F = mean(f^2), MSE_u = mean(g_u^2) + mean(g_K^2) (0 for an
    empty K set), interface terms 0."""
    prob = W.c5_xpinn_inverse_diffusion(seed=0, scale=0.02)
    params = [np.zeros_like(s.params) for s in prob.subdomains]
    terms, _ = O.loss_and_grad(prob, params)
    n_empty = 0
    for q, s in enumerate(prob.subdomains):
        f = s.res_f.astype(np.float64)[:, 0]
        gu = s.bnd_g.astype(np.float64)[:, 0]
        gk = s.aux_g.astype(np.float64)[:, 0]
        ref = (np.mean(gu * gu) if gu.size else 0.0) + (np.mean(gk * gk) if gk.size else 0.0)
        n_empty += gk.size == 0
        assert terms[q, 2] == pytest.approx(np.mean(f * f), rel=1e-13)
        assert terms[q, 1] == pytest.approx(ref, rel=1e-13, abs=1e-300)
        assert terms[q, 3] == 0 and terms[q, 4] == 0
    assert n_empty >= 1   # an interior cell has no K data


def test_inverse_interface_terms():
    """Identical (u, K) pairs on both sides of every interface give zero
    interface terms; the u-average term counts both u and K jumps."""
    prob = _tiny_c5(seed=2)
    p0 = prob.subdomains[0].params
    terms, _ = O.loss_and_grad(prob, [p0.copy() for _ in prob.subdomains])
    assert np.all(terms[:, 3] == 0) and np.all(terms[:, 4] == 0)
    params = [W.perturb_params(s.params, 5, 0.3) for s in prob.subdomains]
    terms, _ = O.loss_and_grad(prob, params)
    e = prob.interfaces[0]
    a, b = prob.subdomains[e.a], prob.subdomains[e.b]
    z = torch.tensor(e.xy, dtype=DT)
    na = W.param_count(a.widths)
    nb = W.param_count(b.widths)
    ta, tb = torch.tensor(params[e.a], dtype=DT), torch.tensor(params[e.b], dtype=DT)
    du = O.mlp(ta[:na], a.widths, z) - O.mlp(tb[:nb], b.widths, z)
    dk = O.mlp(ta[na:], a.aux_widths, z) - O.mlp(tb[nb:], b.aux_widths, z)
    own = float((du ** 2).mean() + (dk ** 2).mean()) / 4
    others = 0.0
    for e2 in prob.interfaces[1:]:
        if e.a in (e2.a, e2.b):
            q2 = e2.b if e2.a == e.a else e2.a
            c = prob.subdomains[q2]
            nc = W.param_count(c.widths)
            tc = torch.tensor(params[q2], dtype=DT)
            z2 = torch.tensor(e2.xy, dtype=DT)
            d1 = O.mlp(ta[:na], a.widths, z2) - O.mlp(tc[:nc], c.widths, z2)
            d2 = O.mlp(ta[na:], a.aux_widths, z2) - O.mlp(tc[nc:], c.aux_widths, z2)
            others += float((d1 ** 2).mean() + (d2 ** 2).mean()) / 4
    assert terms[e.a, 3] == pytest.approx(own + others, rel=1e-12)


def test_inverse_gradient_vs_central_fd():
    prob = _tiny_c5(seed=3, scale=0.008)
    params = [W.perturb_params(s.params, 4, 0.3) for s in prob.subdomains]
    _, grads = O.loss_and_grad(prob, params)
    for q in (0, 3):
        fd = _fd_grad(prob, params, q)
        np.testing.assert_allclose(grads[q], fd, rtol=2e-6, atol=1e-8)
        n_u = W.param_count(prob.subdomains[q].widths)
        assert np.linalg.norm(grads[q][n_u:]) > 1e-6   # the K-network is trained too


def test_inverse_local_gradient_vs_gradient_of_total():
    prob = _tiny_c5(seed=4)
    params = [W.perturb_params(s.params, 1, 0.2) for s in prob.subdomains]
    _, g_local = O.loss_and_grad(prob, params)
    g_total = O.grad_of_total(prob, params)
    prob_i = _tiny_c5(seed=4)
    for s in prob_i.subdomains:
        s.loss_w = (0.0, 0.0, 1.0, 1.0)
    _, g_iface = O.loss_and_grad(prob_i, params)
    for q in range(prob.n_sd):
        np.testing.assert_allclose(g_total[q], g_local[q] + g_iface[q], rtol=1e-10, atol=1e-13)


def test_subdomain_without_points_has_zero_loss_and_gradient():
    """A subdomain with no residual, data or interface points: every mean is
    over an empty set (0), so J_q = 0 and its gradient is 0."""
    prob = W.custom_box_problem("xpinn", "poisson2d", 2, 1, [[2, 4, 4, 1], [2, 3, 1]], [9, 0], n_bnd_seg=0,
                                n_iface=0, seed=1)
    prob.interfaces = []
    terms, grads = O.loss_and_grad(prob, [s.params for s in prob.subdomains])
    assert np.all(terms[1] == 0) and np.all(grads[1] == 0) and grads[1].shape == prob.subdomains[1].params.shape
    assert terms[0, 2] > 0 and np.linalg.norm(grads[0]) > 0


# --------------------------------------------------------------------------
# space-time decomposition of the viscous Burgers problem (Sec. 7.5)


def _tiny_space_time(method, nx, nt, widths=(2, 3, 3, 1), seed=2):
    prob = W.burgers_space_time(method, nx, nt, seed=seed, scale=0.0004, n_iface=300)
    rng = np.random.default_rng(seed)
    for s in prob.subdomains:
        s.widths = list(widths)
        s.params = _rand_theta(rng, s.widths).numpy().astype(np.float32)
    return prob


def _net(prob, params, q, z):
    return O.mlp(torch.tensor(params[q], dtype=DT), prob.subdomains[q].widths, z)[:, 0]


def test_space_time_xpinn_burgers_gradient_vs_central_fd():
    """2 x 2 space-time boxes: subdomain 0 has initial, boundary, a space and
    a time interface; subdomain 3 a space and a time interface from the other
    side."""
    prob = _tiny_space_time("xpinn", 2, 2)
    assert sorted(tuple(e.normal) for e in prob.interfaces) == [(0.0, 1.0), (0.0, 1.0), (1.0, 0.0), (1.0, 0.0)]
    params = [W.perturb_params(s.params, 6, 0.3) for s in prob.subdomains]
    _, grads = O.loss_and_grad(prob, params)
    for q in (0, 3):
        np.testing.assert_allclose(grads[q], _fd_grad(prob, params, q), rtol=2e-6, atol=1e-8)


def test_cpinn_time_interface_flux_is_the_jump_of_u():
    """Across t = const the normal (0, 1) picks the time component u of the
    space-time flux (u^2/2 - nu u_x, u): the flux term is the mean squared
    jump of u, four times the average-solution term, whatever nu and u_x."""
    prob = _tiny_space_time("cpinn", 1, 2)
    params = [s.params for s in prob.subdomains]
    (e,) = prob.interfaces
    z = torch.tensor(e.xy, dtype=DT)
    jump2 = float(((_net(prob, params, 0, z) - _net(prob, params, 1, z)) ** 2).mean())
    terms, _ = O.loss_and_grad(prob, params)
    for q in range(2):
        assert terms[q, 4] == pytest.approx(jump2, rel=1e-12)
        assert terms[q, 3] == pytest.approx(jump2 / 4, rel=1e-12)


def test_xpinn_time_interface_residual_continuity_by_fd():
    """XPINN residual continuity on a time interface: the mean squared jump of
    u_t + u u_x - nu u_xx between the two networks, the derivatives taken by
    central differences of the networks in (x, t)."""
    prob = _tiny_space_time("xpinn", 1, 2, widths=(2, 5, 5, 1))
    params = [W.perturb_params(s.params, 3, 0.2) for s in prob.subdomains]
    (e,) = prob.interfaces
    nu = prob.coef[0]
    z = torch.tensor(e.xy, dtype=DT)

    def burgers_fd(q):
        u = lambda dz: _net(prob, params, q, z + torch.tensor(dz, dtype=DT))
        h1, h2 = 1e-5, 1e-3
        ut = (u([0, h1]) - u([0, -h1])) / (2 * h1)
        ux = (u([h1, 0]) - u([-h1, 0])) / (2 * h1)
        uxx = (u([h2, 0]) - 2 * u([0, 0]) + u([-h2, 0])) / h2 ** 2
        return ut + u([0, 0]) * ux - nu * uxx

    ref = float(((burgers_fd(0) - burgers_fd(1)) ** 2).mean())
    terms, _ = O.loss_and_grad(prob, params)
    assert ref > 0
    for q in range(2):
        assert terms[q, 4] == pytest.approx(ref, rel=1e-5)


# --------------------------------------------------------------------------
# conservative fluxes (Table 1 for Navier-Stokes) and per-interface conditions


@pytest.mark.parametrize("pde,widths,coef", [("poisson2d", [2, 5, 5, 1], ()), ("burgers1d", [2, 5, 5, 1], (0.01 / math.pi,)),
                                             ("ns2d_steady", [2, 6, 5, 3], (40.0,))])
def test_flux_divergence_is_the_residual(pde, widths, coef):
    """div f(u) by central differences of the oracle's normal fluxes along
    n = e_x and n = e_y equals the operator: -Lap u (Poisson), u_t + u u_x -
    nu u_xx (Burgers, inputs (x, t)); for Navier-Stokes the divergence of the
    momentum fluxes of Table 1 is F_1 + u F_3 and F_2 + v F_3, that of the
    mass flux F_3 (f = 0)."""
    rng = np.random.default_rng(8)
    theta = _rand_theta(rng, widths)
    z = torch.tensor(rng.uniform(-0.8, 0.8, (9, 2)), dtype=DT)
    ex, ey = torch.tensor([1.0, 0.0], dtype=DT), torch.tensor([0.0, 1.0], dtype=DT)

    def flux(zz, n):
        return O.normal_flux(pde, coef, O.input_streams(theta, widths, zz, pde, create_graph=False), n)

    h = 1e-5
    div = ((flux(z + h * ex, ex) - flux(z - h * ex, ex)) + (flux(z + h * ey, ey) - flux(z - h * ey, ey))) / (2 * h)
    st = O.input_streams(theta, widths, z, pde, create_graph=False)
    F = O.residual(pde, coef, st, torch.zeros((z.shape[0], 3 if pde == "ns2d_steady" else 1), dtype=DT))
    if pde == "ns2d_steady":
        u, v = st["u"][:, 0], st["u"][:, 1]
        F = torch.stack([F[:, 0] + u * F[:, 2], F[:, 1] + v * F[:, 2], F[:, 2]], 1)
    np.testing.assert_allclose(div.numpy(), F.numpy(), rtol=1e-6, atol=1e-7 * float(F.abs().max()))


def test_ns_cpinn_flux_term_and_gradient():
    """Two Navier-Stokes boxes with cPINN interfaces: the flux term is the
    mean over the interface of the summed squared jumps of the three normal
    fluxes, written out from Table 1 here, and the gradient matches central
    differences."""
    prob = W.custom_box_problem("cpinn", "ns2d_steady", 2, 1, [[2, 4, 3, 3], [2, 3, 4, 3]], [7, 6],
                                n_bnd_seg=3, n_iface=6, seed=6, coef=(40.0,), domain=(-0.5, 1.0, -0.5, 1.5))
    params = [W.perturb_params(s.params, 4, 0.3) for s in prob.subdomains]
    (e,) = prob.interfaces
    nx, ny = (float(c) for c in e.normal)
    z = torch.tensor(e.xy, dtype=DT)

    def table1(q):
        st = O.input_streams(torch.tensor(params[q], dtype=DT), prob.subdomains[q].widths, z, "ns2d_steady",
                             create_graph=False)
        (U, V, P), d = st["u"].T, st["du"]
        re = 40.0
        fxx, fxy = U * U + P - d[:, 0, 0] / re, U * V - d[:, 0, 1] / re
        fyx, fyy = U * V - d[:, 1, 0] / re, V * V + P - d[:, 1, 1] / re
        return torch.stack([nx * fxx + ny * fxy, nx * fyx + ny * fyy, nx * U + ny * V], 1)

    ref = float(((table1(0) - table1(1)) ** 2).sum(1).mean())
    terms, grads = O.loss_and_grad(prob, params)
    assert terms[0, 4] == pytest.approx(ref, rel=1e-12) and terms[1, 4] == pytest.approx(ref, rel=1e-12)
    for q in range(2):
        np.testing.assert_allclose(grads[q], _fd_grad(prob, params, q), rtol=2e-6, atol=1e-8)


def test_hybrid_interfaces_take_each_condition():
    """cPINN across space interfaces, XPINN across time interfaces (2 x 2
    space-time boxes): each subdomain's fourth term is the cPINN flux term of
    its space interface plus the XPINN residual term of its time interface,
    and the gradient matches central differences."""
    hyb = _tiny_space_time("hybrid", 2, 2)
    params = [W.perturb_params(s.params, 7, 0.3) for s in hyb.subdomains]
    kinds = {(e.a, e.b): e.method for e in hyb.interfaces}
    assert kinds == {(0, 1): "cpinn", (0, 2): "xpinn", (1, 3): "xpinn", (2, 3): "cpinn"}
    terms, grads = O.loss_and_grad(hyb, params)
    parts = {}
    for method in ("cpinn", "xpinn"):
        one = _tiny_space_time(method, 2, 2)
        keep = "cpinn" if method == "cpinn" else "xpinn"
        one.interfaces = [e for e, h in zip(one.interfaces, hyb.interfaces) if h.method == keep]
        parts[method], _ = O.loss_and_grad(one, params)
    np.testing.assert_allclose(terms[:, 4], parts["cpinn"][:, 4] + parts["xpinn"][:, 4], rtol=1e-12)
    np.testing.assert_allclose(terms[:, 3], parts["cpinn"][:, 3] + parts["xpinn"][:, 3], rtol=1e-12)
    for q in (0, 3):
        np.testing.assert_allclose(grads[q], _fd_grad(hyb, params, q), rtol=2e-6, atol=1e-8)


# --------------------------------------------------------------------------
# activation choice and trainable slopes (Sec. 3, Table 4)


@pytest.mark.parametrize("act", ["tanh", "sin", "cos"])
def test_adaptive_input_streams_vs_central_fd(act):
    """u, grad u and Lap u of an adaptive network (slopes away from 1/n)
    against central differences of the network itself."""
    rng = np.random.default_rng(12)
    widths = [2, 5, 4, 1]
    theta = torch.cat([_rand_theta(rng, widths), torch.tensor([0.13, 0.07], dtype=DT)])
    z = torch.tensor(rng.uniform(-0.7, 0.7, (6, 2)), dtype=DT)
    st = O.input_streams(theta, widths, z, "poisson2d", create_graph=False, act=act, slope_n=10.0)
    f = lambda zz: O.mlp(theta, widths, zz, act, 10.0)[:, 0]
    h = 1e-4
    e = [torch.tensor([h, 0.0], dtype=DT), torch.tensor([0.0, h], dtype=DT)]
    for i in range(2):
        d1 = (f(z + e[i]) - f(z - e[i])) / (2 * h)
        np.testing.assert_allclose(st["du"][:, 0, i].numpy(), d1.numpy(), rtol=1e-6, atol=1e-8)
    lap = sum((f(z + e[i]) - 2 * f(z) + f(z - e[i])) / h ** 2 for i in range(2))
    np.testing.assert_allclose(st["lap"][:, 0].numpy(), lap.numpy(), rtol=1e-4, atol=1e-5)


def test_activation_closed_forms():
    """One hidden neuron: u = w2 Phi(n a (w1 . z + b1)) + b2 for each Phi."""
    z = torch.tensor([[0.3, -0.2]], dtype=DT)
    w1, b1, w2, b2, a = [0.7, -1.1], 0.25, 1.3, -0.4, 0.15
    theta = torch.tensor(w1 + [b1, w2, b2, a], dtype=DT)
    y = 10.0 * a * (0.7 * 0.3 - 1.1 * -0.2 + 0.25)
    for act, fn in (("tanh", math.tanh), ("sin", math.sin), ("cos", math.cos)):
        u = float(O.mlp(theta, [2, 1, 1], z, act, 10.0)[0, 0])
        assert u == pytest.approx(w2 * fn(y) + b2, rel=1e-14)
    # not adaptive: n a^k = 1
    assert float(O.mlp(theta[:-1], [2, 1, 1], z, "sin")[0, 0]) == pytest.approx(w2 * math.sin(y / (10 * a)) + b2,
                                                                                  rel=1e-14)


def _adaptive_two_box(method, acts, pde="poisson2d", seed=3):
    if pde == "poisson2d":
        prob = W.custom_box_problem(method, pde, 2, 1, [[2, 4, 3, 1], [2, 3, 3, 3, 1]], [9, 8], n_bnd_seg=4,
                                    n_iface=6, seed=seed)
    else:
        prob = W.custom_box_problem(method, pde, 2, 1, [[2, 4, 3, 3], [2, 3, 4, 3]], [7, 6], n_bnd_seg=3,
                                    n_iface=5, seed=seed, coef=(40.0,), domain=(-0.5, 1.0, -0.5, 1.5))
    return W.with_activations(prob, acts)


@pytest.mark.parametrize("method,acts", [("xpinn", ("sin", "cos")), ("cpinn", ("cos", "tanh")),
                                         ("xpinn", ("tanh", "sin"))])
def test_adaptive_gradient_vs_central_fd(method, acts):
    """Gradients of weights, biases and slopes of adaptive networks with
    different activations on the two sides of an interface."""
    prob = _adaptive_two_box(method, acts)
    params = [W.perturb_params(s.params, 5, 0.3) for s in prob.subdomains]
    _, grads = O.loss_and_grad(prob, params)
    for q in range(2):
        assert grads[q].shape == (W.param_count(prob.subdomains[q].widths, True),)
        np.testing.assert_allclose(grads[q], _fd_grad(prob, params, q), rtol=2e-6, atol=1e-8)


def _slope_identity(widths, theta, grad, n_nets_widths=None):
    """a^k dJ/da^k - (<W^k, dJ/dW^k> + <b^k, dJ/db^k>) for every hidden layer
    k of each network (zero: scaling n a^k by lambda equals scaling W^k, b^k)."""
    out, off = [], 0
    for wd in n_nets_widths or [widths]:
        lay = []
        for k in range(1, len(wd)):
            n = wd[k] * wd[k - 1] + wd[k]
            lay.append(slice(off, off + n))
            off += n
        for k in range(len(wd) - 2):
            s = off + k
            out.append((theta[s] * grad[s], float(np.dot(theta[lay[k]], grad[lay[k]]))))
        off += len(wd) - 2
    assert off == theta.size
    return out


@pytest.mark.parametrize("pde,acts", [("poisson2d", ("sin", "cos")), ("ns2d_steady", ("tanh", "cos"))])
def test_slope_gradient_scaling_identity(pde, acts):
    """a^k dJ/da^k = <W^k, dJ/dW^k> + <b^k, dJ/db^k>: the slope scales the
    pre-activation of layer k exactly as a common factor on W^k and b^k."""
    prob = _adaptive_two_box("xpinn", acts, pde=pde)
    params = [W.perturb_params(s.params, 6, 0.3) for s in prob.subdomains]
    _, grads = O.loss_and_grad(prob, params)
    for q in range(2):
        th = params[q].astype(np.float64)
        for lhs, rhs in _slope_identity(prob.subdomains[q].widths, th, grads[q]):
            assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-14)


def test_adaptive_at_initial_slopes_equals_fixed_activation():
    """With n a^k = 1 an adaptive network computes what the fixed network
    computes: same loss terms and the same weight and bias gradients (n = 8
    here, so that a^k = 1/n is exact in float32)."""
    fixed = _two_box("xpinn")
    adapt = W.with_activations(_two_box("xpinn"), ("tanh",), slope_n=8.0)
    tf, gf = O.loss_and_grad(fixed, [s.params for s in fixed.subdomains])
    ta, ga = O.loss_and_grad(adapt, [s.params for s in adapt.subdomains])
    np.testing.assert_allclose(ta, tf, rtol=1e-13)
    for q in range(2):
        n = gf[q].size
        np.testing.assert_allclose(ga[q][:n], gf[q], rtol=1e-12, atol=1e-15)
        assert ga[q].size == n + len(fixed.subdomains[q].widths) - 2


def test_table4_inverse_problem_inputs_and_gradient():
    """The inverse problem with Table 4's networks: activations and residual
    counts as listed; a small instance's gradient (both networks, slopes
    included) against central differences on sampled entries and the slope
    identity for every layer of both networks."""
    full = W.c5_table4_adaptive(seed=0)
    assert [s.act for s in full.subdomains] == list(W.TABLE4_ACTS)
    assert [s.res_xy.shape[0] for s in full.subdomains] == list(W.TABLE4_NRES)
    assert all(s.widths == [2, 80, 80, 80, 1] and s.aux_widths == [2, 80, 80, 80, 1] and s.adaptive
               for s in full.subdomains)
    prob = W.c5_table4_adaptive(seed=1, scale=0.004)
    for s in prob.subdomains:
        s.widths, s.aux_widths = [2, 4, 3, 1], [2, 3, 3, 1]
        rng = np.random.default_rng(2)
        s.params = np.concatenate([W.glorot_params(rng, s.widths, True), W.glorot_params(rng, s.aux_widths, True)])
    params = [W.perturb_params(s.params, 8, 0.3) for s in prob.subdomains]
    _, grads = O.loss_and_grad(prob, params)
    for q in (0, 1, 2):
        sd = prob.subdomains[q]
        idx = list(range(0, params[q].size, 3)) + [params[q].size - 1]
        # J is O(100) here: a wider step keeps the rounding of the differences small
        fd = _fd_grad(prob, params, q, h=1e-5, idx=idx)
        np.testing.assert_allclose(grads[q][idx], fd[idx], rtol=2e-6, atol=1e-7 * np.abs(grads[q]).max())
        for lhs, rhs in _slope_identity(None, params[q].astype(np.float64), grads[q], [sd.widths, sd.aux_widths]):
            assert lhs == pytest.approx(rhs, rel=1e-10, abs=1e-14)


def test_oracle_training_resumes_exactly():
    """Oracle Adam: 3 steps, then 2 more from the returned state, equal 5
    straight steps exactly."""
    prob = _two_box("xpinn", n_res=12)
    p0 = [s.params for s in prob.subdomains]
    ps5, h5 = O.train(prob, p0, 5)
    ps3, h3, st = O.train(prob, p0, 3, return_state=True)
    ps2, h2 = O.train(prob, ps3, 2, state=st)
    for a, b in zip(ps5, ps2):
        assert np.array_equal(a, b)
    assert np.array_equal(h5, np.concatenate([h3, h2]))


# --------------------------------------------------------------------------
# relative L2 error of the stitched solution, and the oracle's training loop


def test_rel_l2_hand_built_vectors():
    """||u - u*|| / ||u*|| on vectors whose ratio is known by construction:
    a scaled copy, an orthogonal perturbation (a Pythagorean triple), and a
    multi-column array taken as one vector (Frobenius norm)."""
    ue = np.array([3.0, 4.0])                      # ||u*|| = 5
    assert O.rel_l2(ue, ue) == 0.0
    assert O.rel_l2(1.2 * ue, ue) == pytest.approx(0.2, rel=1e-15)
    assert O.rel_l2(-ue, ue) == pytest.approx(2.0, rel=1e-15)
    # perturbation (-4, 3) is orthogonal to u* with norm 5: ratio exactly 1,
    # while ||u|| / ||u*|| - 1 would give sqrt(2) - 1
    assert O.rel_l2(ue + np.array([-4.0, 3.0]), ue) == pytest.approx(1.0, rel=1e-15)
    # two columns (u, K): the error is over all entries together
    ue2 = np.array([[1.0, 2.0], [2.0, 4.0]])       # ||u*||_F = 5
    d = np.array([[0.0, 1.0], [0.0, 0.0]])
    assert O.rel_l2(ue2 + d, ue2) == pytest.approx(0.2, rel=1e-15)
    # per-column errors would differ (0 and 1/sqrt(20)); the whole-array value does not
    assert O.rel_l2((ue2 + d)[:, 0], ue2[:, 0]) == 0.0


def test_oracle_train_matches_torch_adam_per_subdomain():
    """The oracle's training loop against torch.optim.Adam, one optimiser per
    subdomain with that subdomain's learning rate, fed the oracle's gradient at
    the current parameters: steps t = 1, 2, 3 straight, then a resume from the
    returned state (t0 = 3) for two more.  An offset in the step index t of
    the bias correction, a shared learning rate or a history entry taken after
    the update fails it."""
    prob = _two_box("xpinn", n_res=12)
    prob.subdomains[0].lr = 2e-2
    prob.subdomains[1].lr = 5e-3
    p0 = [s.params.astype(np.float64) for s in prob.subdomains]
    tp = [torch.tensor(p.copy(), dtype=DT, requires_grad=True) for p in p0]
    opts = [torch.optim.Adam([t], lr=s.lr, betas=(0.9, 0.999), eps=1e-8) for t, s in zip(tp, prob.subdomains)]
    ref_hist = []
    ref_params = []
    for step in range(5):
        cur = [t.detach().numpy().copy() for t in tp]
        terms, grads = O.loss_and_grad(prob, cur)
        ref_hist.append(terms)
        for q in range(2):
            tp[q].grad = torch.tensor(grads[q], dtype=DT)
            opts[q].step()
        ref_params.append([t.detach().numpy().copy() for t in tp])
    ps3, h3, st = O.train(prob, p0, 3, return_state=True)
    assert st[2] == 3
    for q in range(2):
        np.testing.assert_allclose(ps3[q], ref_params[2][q], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(h3, np.stack(ref_hist[:3]), rtol=1e-12, atol=1e-15)
    ps5, h2, st5 = O.train(prob, ps3, 2, state=st, return_state=True)
    assert st5[2] == 5
    for q in range(2):
        np.testing.assert_allclose(ps5[q], ref_params[4][q], rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(h2, np.stack(ref_hist[3:]), rtol=1e-12, atol=1e-15)
    # the steps really moved the parameters by more than the tolerance
    assert min(np.abs(ps5[q] - p0[q]).max() for q in range(2)) > 1e-4


def test_oracle_train_step_index_offset_is_detected():
    """Planted mistake (on the CPU): an Adam loop whose bias correction uses
    t + 1 instead of t departs from torch.optim.Adam at the tolerance of the
    test above, so that test would catch it."""
    rng = np.random.default_rng(3)
    th0 = rng.normal(size=25)
    gs = [rng.normal(size=25) for _ in range(3)]
    p = torch.tensor(th0.copy(), dtype=DT, requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    th, m, v = th0.copy(), np.zeros(25), np.zeros(25)
    for t, g in enumerate(gs, start=1):
        p.grad = torch.tensor(g, dtype=DT)
        opt.step()
        th, m, v = O.adam_step(th, m, v, g, t + 1, 1e-2)
    assert np.abs(th - p.detach().numpy()).max() > 1e-5
