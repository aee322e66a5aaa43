"""FP64 CPU oracle for one domain-decomposed PINN training step.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this module;
only the tests, the smoke check and the CPU-baseline leg of the benchmark do.

It computes, from the plain definitions and in float64 (inputs and parameters
are the float32 values the GPU sees, converted exactly):

* the network of Sec. 3: N^1 = W^1 z + b^1, N^k = W^k Phi(n a^{k-1} N^{k-1}) + b^k,
  identity output layer; Phi is tanh, sin or cos (chosen per subdomain, Table
  4), and the layer-wise slopes a^k are trainable parameters when the network
  is adaptive (else n a^k = 1);
* input derivatives of the network output by automatic differentiation, as the
  paper does for the PDE residual (Sec. 4.1);
* the residual F = L_x(u) - f of Eq. ProSet for the Poisson, Burgers (Eq. BE)
  and steady Navier-Stokes (Eq. NSEq) operators, and for the inverse
  diffusion problem of Eq. heq, div(K grad u) = f, where the conductivity K is
  a second network of the subdomain (Sec. 7.6);
* the per-subdomain losses J(Theta_q) of Eq. cPINNLoss (data, residual,
  average-solution and normal-flux terms) and Eq. XPINNLoss (data, residual,
  average-solution and residual-continuity terms);
* the gradient dJ(Theta_q)/dTheta_q with the neighbour's interface values held
  fixed, as in Algorithm 1 where each rank minimises its own loss using values
  received from its neighbours;
* one Adam step per subdomain (Sec. 6; Kingma-Ba form, beta=(0.9,0.999),
  eps=1e-8);
* the stitched solution of Eq. FSol with the 1/S indicator on interfaces
  (for the inverse problem both u and K are stitched).

Plain PyTorch CPU ops in float64 serve as the library primitives (matmul, tanh,
reverse-mode differentiation).  There is no blocking, fusion or reordering.
"""
from __future__ import annotations

import math
import numpy as np
import torch

DT = torch.float64

POISSON2D = "poisson2d"
BURGERS1D = "burgers1d"
NS2D = "ns2d_steady"
DIFF_INV = "diffusion2d_inv"


# ----------------------------------------------------------------------------
# network (Sec. 3)


ACTIVATIONS = {"tanh": torch.tanh, "sin": torch.sin, "cos": torch.cos}


def n_slopes(widths, slope_n):
    """Trainable slopes of a network: one per hidden layer when adaptive."""
    return len(widths) - 2 if slope_n is not None else 0


def unpack(theta, widths, slope_n=None):
    """Split a flat parameter vector into [(W^k, b^k)], W^k of shape
    (N_k, N_{k-1}), and the slopes a^1..a^{L-1} that follow the layers of an
    adaptive network (None otherwise)."""
    out, off = [], 0
    for k in range(1, len(widths)):
        nin, nout = widths[k - 1], widths[k]
        W = theta[off:off + nout * nin].reshape(nout, nin)
        off += nout * nin
        b = theta[off:off + nout]
        off += nout
        out.append((W, b))
    ns = n_slopes(widths, slope_n)
    slopes = theta[off:off + ns] if ns else None
    off += ns
    assert off == theta.shape[0], (off, theta.shape)
    return out, slopes


def mlp(theta, widths, z, act="tanh", slope_n=None):
    """N^L(z; Theta): Phi(n a^k x) on hidden layer k (n a^k = 1 unless the
    network is adaptive, slope_n = n), identity on the last layer."""
    layers, slopes = unpack(theta, widths, slope_n)
    phi = ACTIVATIONS[act]
    h = z
    for k, (W, b) in enumerate(layers):
        a = h @ W.T + b
        if k < len(layers) - 1:
            if slopes is not None:
                a = (slope_n * slopes[k]) * a
            h = phi(a)
        else:
            h = a
    return h


def net_kw(sd, which="u"):
    """Activation keywords of a subdomain's network ("u", or "K" for the
    conductivity network of the inverse problem, which shares the choice)."""
    act = getattr(sd, "act", "tanh")
    n = getattr(sd, "slope_n", 10.0) if getattr(sd, "adaptive", False) else None
    return {"act": act, "slope_n": n}


def second_order_set(pde):
    """Input directions whose pure second derivatives the operator needs."""
    if pde == BURGERS1D:
        return (0,)          # u_xx only (inputs are (x, t))
    return (0, 1)            # Laplacian in (x, y)


def input_streams(theta, widths, z, pde, create_graph=True, act="tanh", slope_n=None):
    """u, grad u and the second-order sum  sum_{i in S} d^2 u / dz_i^2  per
    output component, by reverse-mode automatic differentiation w.r.t. z."""
    z = z.detach().clone().requires_grad_(True)
    u = mlp(theta, widths, z, act, slope_n)        # (N, D_o)
    n_out = u.shape[1]
    grads, lap = [], []
    S = second_order_set(pde)
    for c in range(n_out):
        g, = torch.autograd.grad(u[:, c].sum(), z, create_graph=True)
        grads.append(g)
        acc = torch.zeros_like(u[:, c])
        for i in S:
            gi, = torch.autograd.grad(g[:, i].sum(), z, create_graph=True)
            acc = acc + gi[:, i]
        lap.append(acc)
    st = {"u": u, "du": torch.stack(grads, 1), "lap": torch.stack(lap, 1)}
    if not create_graph:
        st = {k: v.detach() for k, v in st.items()}
    return st


# ----------------------------------------------------------------------------
# operators (Eq. ProSet: F = L_x(u) - f)


def residual(pde, coef, st, f):
    """F per residual equation, shape (N, n_eq).

    Poisson:  -Lap u - f.
    Burgers:  u_t + u u_x - nu u_xx     (inputs (x, t); f = 0).
    NS:       u u_x + v u_y + p_x - Lap u / Re,
              u v_x + v v_y + p_y - Lap v / Re,
              u_x + v_y.
    """
    u, du, lap = st["u"], st["du"], st["lap"]
    if pde == POISSON2D:
        return (-lap[:, 0] - f[:, 0])[:, None]
    if pde == BURGERS1D:
        nu = coef[0]
        return (du[:, 0, 1] + u[:, 0] * du[:, 0, 0] - nu * lap[:, 0] - f[:, 0])[:, None]
    if pde == NS2D:
        re = coef[0]
        U, V = u[:, 0], u[:, 1]
        F1 = U * du[:, 0, 0] + V * du[:, 0, 1] + du[:, 2, 0] - lap[:, 0] / re - f[:, 0]
        F2 = U * du[:, 1, 0] + V * du[:, 1, 1] + du[:, 2, 1] - lap[:, 1] / re - f[:, 1]
        F3 = du[:, 0, 0] + du[:, 1, 1] - f[:, 2]
        return torch.stack([F1, F2, F3], 1)
    raise ValueError(pde)


def residual_inverse(stu, stk, f):
    """Eq. heq with the divergence expanded: F = K Lap u + K_x u_x + K_y u_y - f,
    from the u-network streams stu and the K-network streams stk; (N, 1)."""
    K, dK = stk["u"][:, 0], stk["du"][:, 0]
    du, lap = stu["du"][:, 0], stu["lap"][:, 0]
    return (K * lap + dK[:, 0] * du[:, 0] + dK[:, 1] * du[:, 1] - f[:, 0])[:, None]


def split_theta(prob, q, theta):
    """(solution-network params, K-network params or None) of subdomain q."""
    sd = prob.subdomains[q]
    if sd.aux_widths is None:
        return theta, None
    n = sum(sd.widths[k] * sd.widths[k - 1] + sd.widths[k] for k in range(1, len(sd.widths)))
    n += n_slopes(sd.widths, net_kw(sd)["slope_n"])
    return theta[:n], theta[n:]


def normal_flux(pde, coef, st, n):
    """f(u) . n for the conservative form of the equation, shape (N, n_eq).

    Poisson:  f = -grad u.
    Burgers:  space-time flux (u^2/2 - nu u_x, u) of u_t + (u^2/2 - nu u_x)_x = 0.
    NS:       the x-momentum, y-momentum and mass fluxes of Table 1, with
              (x, y) components
              (u^2 + p - u_x/Re, uv - u_y/Re),
              (uv - v_x/Re, v^2 + p - v_y/Re),
              (u, v).
    """
    u, du = st["u"], st["du"]
    if pde == POISSON2D:
        return (-(n[0] * du[:, 0, 0] + n[1] * du[:, 0, 1]))[:, None]
    if pde == BURGERS1D:
        nu = coef[0]
        fx = 0.5 * u[:, 0] ** 2 - nu * du[:, 0, 0]
        return (n[0] * fx + n[1] * u[:, 0])[:, None]
    if pde == NS2D:
        re = coef[0]
        U, V, P = u[:, 0], u[:, 1], u[:, 2]
        mx = n[0] * (U * U + P - du[:, 0, 0] / re) + n[1] * (U * V - du[:, 0, 1] / re)
        my = n[0] * (U * V - du[:, 1, 0] / re) + n[1] * (V * V + P - du[:, 1, 1] / re)
        ms = n[0] * U + n[1] * V
        return torch.stack([mx, my, ms], 1)
    raise NotImplementedError(f"cPINN flux for {pde}")


# ----------------------------------------------------------------------------
# losses (Eqs. cPINNLoss, XPINNLoss)


def _t(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float64), dtype=DT)


def _mean_sq(x):
    """(1/N) sum_i sum_c x_ic^2; an empty set contributes 0."""
    if x.shape[0] == 0:
        return torch.zeros((), dtype=DT)
    return (x ** 2).sum() / x.shape[0]


def interface_method(prob, e):
    """The interface condition of e: its own method where one is set (the
    cPINN-in-space, XPINN-in-time combination of the conclusions), else the
    problem's."""
    return getattr(e, "method", None) or prob.method


def interface_value(prob, q, theta, e, create_graph):
    """What subdomain q contributes on interface e: u, and flux.n (cPINN) or F (XPINN)."""
    sd = prob.subdomains[q]
    z = _t(e.xy)
    method = interface_method(prob, e)
    if prob.pde == DIFF_INV:
        # the pair (u, K) is the solution whose average is matched; the
        # operator value L(u, K) = div(K grad u) is compared (f cancels)
        if method != "xpinn":
            raise NotImplementedError("the inverse problem uses XPINN interfaces")
        thu, thk = split_theta(prob, q, theta)
        stu = input_streams(thu, sd.widths, z, prob.pde, create_graph=create_graph, **net_kw(sd))
        stk = input_streams(thk, sd.aux_widths, z, prob.pde, create_graph=create_graph, **net_kw(sd, "K"))
        f0 = torch.zeros((z.shape[0], 1), dtype=DT)
        return torch.cat([stu["u"], stk["u"]], 1), residual_inverse(stu, stk, f0)
    st = input_streams(theta, sd.widths, z, prob.pde, create_graph=create_graph, **net_kw(sd))
    u = st["u"]
    if method == "cpinn":
        other = normal_flux(prob.pde, prob.coef, st, _t(e.normal))
    else:
        # the forcing f is the same on both sides of a common point and cancels
        # in F_q - F_q+; zero is passed so only L_x(u) is compared
        f0 = torch.zeros((z.shape[0], prob.n_eq), dtype=DT)
        other = residual(prob.pde, prob.coef, st, f0)
    return u, other


def subdomain_terms(prob, q, thetas, grad_mode="local"):
    """[J, MSE_u, MSE_F, MSE_uavg, MSE_flux | MSE_R] for subdomain q.

    grad_mode 'local': neighbour values are constants (what each rank sees after
    the exchange of Algorithm 1).  'sum' keeps neighbours differentiable (used
    only by tests of the alternative readings)."""
    sd = prob.subdomains[q]
    th = thetas[q]
    thu, thk = split_theta(prob, q, th)
    Wu, WF, WI, W4 = sd.loss_w
    # data / boundary term (for the inverse problem also the K data; the two
    # mean squares are summed like the components of a vector solution)
    if sd.bnd_xy.shape[0] > 0:
        ub = mlp(thu, sd.widths, _t(sd.bnd_xy), **net_kw(sd))
        mse_u = _mean_sq(ub - _t(sd.bnd_g))
    else:
        mse_u = torch.zeros((), dtype=DT)
    if thk is not None and sd.aux_xy.shape[0] > 0:
        kb = mlp(thk, sd.aux_widths, _t(sd.aux_xy), **net_kw(sd, "K"))
        mse_u = mse_u + _mean_sq(kb - _t(sd.aux_g))
    # residual term
    if sd.res_xy.shape[0] > 0:
        st = input_streams(thu, sd.widths, _t(sd.res_xy), prob.pde, **net_kw(sd))
        if thk is None:
            F = residual(prob.pde, prob.coef, st, _t(sd.res_f))
        else:
            stk = input_streams(thk, sd.aux_widths, _t(sd.res_xy), prob.pde, **net_kw(sd, "K"))
            F = residual_inverse(st, stk, _t(sd.res_f))
        mse_f = _mean_sq(F)
    else:
        mse_f = torch.zeros((), dtype=DT)
    # interface terms, summed over the neighbours q+ of q
    mse_avg = torch.zeros((), dtype=DT)
    mse_4 = torch.zeros((), dtype=DT)
    for e in prob.interfaces:
        if q not in (e.a, e.b):
            continue
        nb = e.b if q == e.a else e.a
        uq, oq = interface_value(prob, q, th, e, create_graph=True)
        th_nb = thetas[nb] if grad_mode == "sum" else thetas[nb].detach()
        un, on = interface_value(prob, nb, th_nb, e, create_graph=(grad_mode == "sum"))
        uavg = 0.5 * (uq + un)
        mse_avg = mse_avg + _mean_sq(uq - uavg)
        mse_4 = mse_4 + _mean_sq(oq - on)
    J = Wu * mse_u + WF * mse_f + WI * mse_avg + W4 * mse_4
    return torch.stack([J, mse_u, mse_f, mse_avg, mse_4])


def loss_and_grad(prob, params, grad_mode="local"):
    """Loss terms (n_sd, 5) and per-subdomain gradients dJ_q/dTheta_q (float64)."""
    thetas = [_t(p).requires_grad_(True) for p in params]
    terms, grads = [], []
    for q in range(prob.n_sd):
        t = subdomain_terms(prob, q, thetas, grad_mode=grad_mode)
        if grad_mode == "sum":
            terms.append(t.detach().numpy())
            grads.append(None)
            continue
        if t[0].requires_grad:
            g, = torch.autograd.grad(t[0], thetas[q], allow_unused=True)
        else:
            g = None   # no points at all: J_q is the constant 0 (empty means are 0)
        if g is None:
            g = torch.zeros_like(thetas[q])
        terms.append(t.detach().numpy())
        grads.append(g.detach().numpy())
    return np.stack(terms), grads


def grad_of_total(prob, params):
    """Gradient of sum_r J_r w.r.t. every Theta_q (rejected reading; tests only)."""
    thetas = [_t(p).requires_grad_(True) for p in params]
    total = sum(subdomain_terms(prob, q, thetas, grad_mode="sum")[0] for q in range(prob.n_sd))
    gs = torch.autograd.grad(total, thetas, allow_unused=True)
    return [(g if g is not None else torch.zeros_like(t)).detach().numpy() for g, t in zip(gs, thetas)]


# ----------------------------------------------------------------------------
# optimiser (Sec. 6)


def adam_step(theta, m, v, g, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; t is the 1-based index of this step."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    theta = theta - lr * mhat / (np.sqrt(vhat) + eps)
    return theta, m, v


def train(prob, params, n_steps, round_to_f32=False, state=None, return_state=False):
    """n_steps of (loss_and_grad, Adam) per subdomain; returns params and loss
    history (and the Adam state (m, v, t) with return_state).  state resumes
    from an Adam state returned earlier."""
    ps = [np.asarray(p, np.float64) for p in params]
    if state is None:
        ms = [np.zeros_like(p) for p in ps]
        vs = [np.zeros_like(p) for p in ps]
        t0 = 0
    else:
        ms, vs, t0 = [m.copy() for m in state[0]], [v.copy() for v in state[1]], state[2]
    hist = []
    for t in range(t0 + 1, t0 + n_steps + 1):
        feed = [p.astype(np.float32) for p in ps] if round_to_f32 else ps
        terms, grads = loss_and_grad(prob, feed)
        hist.append(terms)
        for q in range(prob.n_sd):
            ps[q], ms[q], vs[q] = adam_step(ps[q], ms[q], vs[q], grads[q], t, prob.subdomains[q].lr)
    if return_state:
        return ps, np.stack(hist), (ms, vs, t0 + n_steps)
    return ps, np.stack(hist)


# ----------------------------------------------------------------------------
# stitched solution (Eq. FSol) and error


def eval_stitched(prob, params, xy, owner):
    """u(z) = sum_q u_q(z) 1_{Omega_q}(z), indicator 1/S on common interfaces.

    owner[i] lists the S subdomains whose closure holds point i (-1 padded)."""
    xy = np.asarray(xy)
    inv = prob.pde == DIFF_INV
    out = np.zeros((xy.shape[0], prob.d_out + (1 if inv else 0)))
    cnt = (owner >= 0).sum(1)
    with torch.no_grad():
        for q in range(prob.n_sd):
            sel = np.nonzero((owner == q).any(1))[0]
            if sel.size == 0:
                continue
            sd = prob.subdomains[q]
            thu, thk = split_theta(prob, q, _t(params[q]))
            u = mlp(thu, sd.widths, _t(xy[sel]), **net_kw(sd)).numpy()
            if inv:   # inverse problem: columns (u, K)
                u = np.concatenate([u, mlp(thk, sd.aux_widths, _t(xy[sel]), **net_kw(sd, "K")).numpy()], 1)
            out[sel] += u / cnt[sel][:, None]
    return out


def rel_l2(u, u_exact):
    return float(np.linalg.norm(u - u_exact) / np.linalg.norm(u_exact))
