"""Seeded synthetic workloads for domain-decomposed PINN training.

This module only *generates inputs*: subdomain geometry, point sets, forcing
and target values from closed-form fields, and Glorot-initialised parameters.
It holds none of the method's arithmetic (no network, residual, loss, gradient
or optimiser); both the FP64 oracle and the HIP path consume what it returns.

Problem structure follows Sec. 4.2 (non-overlapping subdomains, one network
each, residual / training / interface point sets per subdomain) and the
pre-processing stage of Sec. 5.1 (domain split, per-subdomain point sets, an
edge -> interface-points table). The concrete shapes follow the paper's
experiments: the 2D Poisson manufactured problem, the 1D viscous Burgers
equation of Sec. 7.3/7.5 (Eq. BE), and steady incompressible Navier-Stokes
(Eq. NSEq, Kovasznay closed form standing in for the cavity data), the inverse
diffusion problem of Sec. 7.6 (Eq. heq) with a seeded star domain and Voronoi
cells standing in for the US map.

Randomness: numpy PCG64 through ``SeedSequence(seed).spawn(4)``; one stream
each for geometry, points, parameters and observation noise.  Coordinates and
targets are produced in float64 and rounded once to float32; everything
downstream (oracle and GPU) sees the identical float32 values.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math
import numpy as np

METHOD_CPINN = "cpinn"
METHOD_XPINN = "xpinn"

PDE_POISSON2D = "poisson2d"
PDE_BURGERS1D = "burgers1d"
PDE_NS2D = "ns2d_steady"
PDE_DIFFUSION2D_INV = "diffusion2d_inv"

#: number of residual equations / network outputs per PDE
PDE_NEQ = {PDE_POISSON2D: 1, PDE_BURGERS1D: 1, PDE_NS2D: 3, PDE_DIFFUSION2D_INV: 1}
PDE_DOUT = {PDE_POISSON2D: 1, PDE_BURGERS1D: 1, PDE_NS2D: 3, PDE_DIFFUSION2D_INV: 1}


@dataclass
class Subdomain:
    """One subdomain Omega_q with its own network (Sec. 4.2)."""
    widths: list            # N_0 .. N_L of the solution network
    loss_w: tuple           # (W_u, W_F, W_I, W_flux | W_IF)  (Eqs. cPINNLoss / XPINNLoss)
    lr: float               # per-subdomain Adam learning rate (Sec. 6)
    res_xy: np.ndarray      # (N_F, 2) float32 residual points
    res_f: np.ndarray       # (N_F, n_eq) float32 forcing f(x) at residual points
    bnd_xy: np.ndarray      # (N_u, 2) float32 training (boundary/initial/data) points
    bnd_g: np.ndarray       # (N_u, D_o) float32 targets u^(i)
    params: np.ndarray      # flat float32, per layer W[out][in] row-major then b[out]
    # second network (inverse problems only: the unknown coefficient K); its
    # parameters follow the solution network's in `params`
    aux_widths: list | None = None
    aux_xy: np.ndarray | None = None     # (N_K, 2) points with known K values
    aux_g: np.ndarray | None = None      # (N_K, 1) K targets
    # activation of the subdomain's networks (Sec. 3, Table 4): Phi in
    # {"tanh", "sin", "cos"} applied to n a^k x on hidden layer k; adaptive
    # networks train the slopes a^k (one per hidden layer, stored after the
    # layers of each network, initialised to n a^k = 1), else n a^k = 1
    act: str = "tanh"
    adaptive: bool = False
    slope_n: float = 10.0


@dataclass
class Interface:
    """Common interface between Omega_a and Omega_b with its points (Sec. 5.1)."""
    a: int
    b: int
    xy: np.ndarray          # (N_e, 2) float32
    normal: np.ndarray      # (2,) float32 unit normal pointing from a to b
    # interface condition of this interface ("cpinn" flux or "xpinn" residual
    # continuity); None: the problem's method
    method: str | None = None


@dataclass
class Problem:
    name: str
    method: str
    pde: str
    coef: tuple             # (nu,) for Burgers, (Re,) for NS, () otherwise
    subdomains: list
    interfaces: list
    eval_xy: np.ndarray = None      # (n, 2) float32 evaluation grid
    eval_owner: np.ndarray = None   # (n, 4) int32 subdomains containing the point, -1 padded
    eval_exact: np.ndarray = None   # (n, D_o) float64 exact solution on the grid
    meta: dict = field(default_factory=dict)

    @property
    def n_sd(self):
        return len(self.subdomains)

    @property
    def d_out(self):
        return PDE_DOUT[self.pde]

    @property
    def n_eq(self):
        return PDE_NEQ[self.pde]

    def n_residual(self):
        return int(sum(s.res_xy.shape[0] for s in self.subdomains))


# ----------------------------------------------------------------------------
# parameters


def param_count(widths, adaptive=False):
    """Parameters of one network: per layer W and b, then one slope per
    hidden layer when adaptive."""
    n = sum(widths[k] * widths[k - 1] + widths[k] for k in range(1, len(widths)))
    return int(n + (len(widths) - 2 if adaptive else 0))


def glorot_params(rng, widths, adaptive=False, slope_n=10.0):
    """Glorot-normal weights, zero biases, flat canonical layout; an adaptive
    network's slopes start at a^k = 1/n (n a^k = 1, Sec. 3)."""
    out = []
    for k in range(1, len(widths)):
        fan_in, fan_out = widths[k - 1], widths[k]
        std = math.sqrt(2.0 / (fan_in + fan_out))
        out.append(rng.normal(0.0, std, size=(fan_out, fan_in)).ravel())
        out.append(np.zeros(fan_out))
    if adaptive:
        out.append(np.full(len(widths) - 2, 1.0 / slope_n))
    return np.concatenate(out).astype(np.float32)


def perturb_params(params, seed, scale=0.05):
    """A seeded relative perturbation, used to test away from initialisation."""
    rng = np.random.default_rng(seed)
    p = params.astype(np.float64)
    return (p + scale * rng.standard_normal(p.shape) * (np.abs(p) + 0.05)).astype(np.float32)


# ----------------------------------------------------------------------------
# closed-form fields


def poisson_exact(x, y):
    return np.sin(np.pi * x) * np.sin(np.pi * y)


def poisson_forcing(x, y):
    # -Lap(sin(pi x) sin(pi y)) = 2 pi^2 sin(pi x) sin(pi y)
    return 2.0 * np.pi ** 2 * np.sin(np.pi * x) * np.sin(np.pi * y)


def kovasznay_lambda(re):
    return 0.5 * re - math.sqrt(0.25 * re * re + 4.0 * math.pi ** 2)


def kovasznay_exact(x, y, re):
    lam = kovasznay_lambda(re)
    e = np.exp(lam * x)
    u = 1.0 - e * np.cos(2 * np.pi * y)
    v = lam / (2 * np.pi) * e * np.sin(2 * np.pi * y)
    p = 0.5 * (1.0 - np.exp(2 * lam * x))
    return np.stack([u, v, p], axis=-1)


def diffusion_fields(x, y):
    """Manufactured u and K for the inverse problem, with f = div(K grad u)."""
    pi = np.pi
    u = np.sin(pi * x) * np.sin(pi * y)
    ux = pi * np.cos(pi * x) * np.sin(pi * y)
    uy = pi * np.sin(pi * x) * np.cos(pi * y)
    lap = -2 * pi * pi * u
    K = 1.0 + 0.5 * np.sin(2 * pi * x) * np.cos(2 * pi * y)
    Kx = pi * np.cos(2 * pi * x) * np.cos(2 * pi * y)
    Ky = -pi * np.sin(2 * pi * x) * np.sin(2 * pi * y)
    f = K * lap + Kx * ux + Ky * uy
    return u, K, f


# ----------------------------------------------------------------------------
# sampling helpers


def _box_points(rng, n, x0, x1, y0, y1):
    return np.stack([rng.uniform(x0, x1, n), rng.uniform(y0, y1, n)], axis=1)


def _segment_points(rng, n, p0, p1):
    s = rng.uniform(0.0, 1.0, n)
    p0 = np.asarray(p0, float)
    p1 = np.asarray(p1, float)
    return p0[None, :] + s[:, None] * (p1 - p0)[None, :]


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64).astype(np.float32))


def _box_grid_problem(name, method, pde, coef, rng_geo, rng_pts, rng_par,
                      xs, ys, widths_fn, nres_fn, n_bnd_seg, n_iface, exact_fn,
                      forcing_fn, loss_w, lr, eval_shape):
    """Cartesian decomposition: boxes [xs[i],xs[i+1]] x [ys[j],ys[j+1]],
    q = j * nx + i (row-major), Dirichlet data on the outer boundary."""
    nx, ny = len(xs) - 1, len(ys) - 1
    d_out = PDE_DOUT[pde]
    n_eq = PDE_NEQ[pde]
    subs = []
    for j in range(ny):
        for i in range(nx):
            q = j * nx + i
            widths = widths_fn(rng_geo, q)
            n_res = nres_fn(rng_geo, q)
            x0, x1, y0, y1 = xs[i], xs[i + 1], ys[j], ys[j + 1]
            res = _box_points(rng_pts, n_res, x0, x1, y0, y1)
            f = forcing_fn(res[:, 0], res[:, 1]).reshape(n_res, n_eq)
            segs = []
            if j == 0:
                segs.append(((x0, y0), (x1, y0)))
            if j == ny - 1:
                segs.append(((x0, y1), (x1, y1)))
            if i == 0:
                segs.append(((x0, y0), (x0, y1)))
            if i == nx - 1:
                segs.append(((x1, y0), (x1, y1)))
            bpts = [_segment_points(rng_pts, n_bnd_seg, a, b) for a, b in segs]
            bnd = np.concatenate(bpts, 0) if bpts else np.zeros((0, 2))
            g = exact_fn(bnd[:, 0], bnd[:, 1]).reshape(len(bnd), d_out)
            subs.append(Subdomain(widths=widths, loss_w=tuple(loss_w), lr=lr,
                                  res_xy=_f32(res), res_f=_f32(f), bnd_xy=_f32(bnd),
                                  bnd_g=_f32(g), params=glorot_params(rng_par, widths)))
    ifaces = []
    for j in range(ny):
        for i in range(nx):
            q = j * nx + i
            if i + 1 < nx:   # vertical edge x = xs[i+1] between q and q+1
                pts = _segment_points(rng_pts, n_iface, (xs[i + 1], ys[j]), (xs[i + 1], ys[j + 1]))
                ifaces.append(Interface(q, q + 1, _f32(pts), _f32([1.0, 0.0])))
            if j + 1 < ny:   # horizontal edge y = ys[j+1] between q and q+nx
                pts = _segment_points(rng_pts, n_iface, (xs[i], ys[j + 1]), (xs[i + 1], ys[j + 1]))
                ifaces.append(Interface(q, q + nx, _f32(pts), _f32([0.0, 1.0])))
    # evaluation grid with the subdomains whose closed box holds each point
    gx = np.linspace(xs[0], xs[-1], eval_shape[0])
    gy = np.linspace(ys[0], ys[-1], eval_shape[1])
    X, Y = np.meshgrid(gx, gy, indexing="ij")
    exy = np.stack([X.ravel(), Y.ravel()], 1)
    exy32 = _f32(exy)
    ex = exy32.astype(np.float64)
    owner = -np.ones((len(ex), 4), np.int32)
    cnt = np.zeros(len(ex), np.int32)
    for j in range(ny):
        for i in range(nx):
            q = j * nx + i
            inside = ((ex[:, 0] >= xs[i]) & (ex[:, 0] <= xs[i + 1]) &
                      (ex[:, 1] >= ys[j]) & (ex[:, 1] <= ys[j + 1]))
            idx = np.nonzero(inside)[0]
            owner[idx, cnt[idx]] = q
            cnt[idx] += 1
    exact = exact_fn(ex[:, 0], ex[:, 1]).reshape(len(ex), d_out)
    return Problem(name=name, method=method, pde=pde, coef=tuple(coef), subdomains=subs,
                   interfaces=ifaces, eval_xy=exy32, eval_owner=owner, eval_exact=exact)


# ----------------------------------------------------------------------------
# the five workloads


def _streams(seed):
    ss = np.random.SeedSequence(seed).spawn(4)
    return [np.random.default_rng(s) for s in ss]


def c1_cpinn_poisson(seed=0, scale=1.0):
    """cPINN, -Lap u = f on [0,1]^2 with u = sin(pi x) sin(pi y), 2x2 boxes,
    nets 2-20-20-20-1, 1000 residual points per box, 50 boundary points per
    outer edge segment, 100 points per interface."""
    g, p, w, _ = _streams(seed)
    n_res = max(1, int(round(1000 * scale)))
    n_b = max(1, int(round(50 * scale)))
    n_i = max(1, int(round(100 * scale)))
    return _box_grid_problem(
        "c1_cpinn_poisson", METHOD_CPINN, PDE_POISSON2D, (), g, p, w,
        [0.0, 0.5, 1.0], [0.0, 0.5, 1.0],
        lambda r, q: [2, 20, 20, 20, 1], lambda r, q: n_res, n_b, n_i,
        poisson_exact, poisson_forcing, (1.0, 1.0, 1.0, 1.0), 1e-3, (201, 201))


def c2_xpinn_poisson(seed=0, scale=1.0):
    """XPINN, same Poisson problem on 4x4 boxes of side 0.25; per subdomain a
    width from {20,40,60,80}, 3..6 hidden layers, and U_int[2000,20000]
    residual points; 50 boundary points per outer segment, 200 per interface."""
    g, p, w, _ = _streams(seed)

    def widths(r, q):
        wd = int(r.choice([20, 40, 60, 80]))
        depth = int(r.integers(3, 7))
        return [2] + [wd] * depth + [1]

    def nres(r, q):
        return max(1, int(round(int(r.integers(2000, 20001)) * scale)))

    n_b = max(1, int(round(50 * scale)))
    n_i = max(1, int(round(200 * scale)))
    cuts = [0.0, 0.25, 0.5, 0.75, 1.0]
    return _box_grid_problem(
        "c2_xpinn_poisson", METHOD_XPINN, PDE_POISSON2D, (), g, p, w, cuts, cuts,
        widths, nres, n_b, n_i, poisson_exact, poisson_forcing,
        (1.0, 1.0, 1.0, 1.0), 1e-3, (201, 201))


def c3_cpinn_burgers(seed=0, scale=1.0, n_strips=8):
    """cPINN, u_t + u u_x = nu u_xx, nu = 0.01/pi, x in [-1,1], t in [0,1],
    u(0,x) = -sin(pi x), u(t,+-1) = 0; n_strips spatial strips; nets
    2-50x6-1; 5000 residual, 256 initial, 100 boundary (end strips) and
    200 interface points.  Inputs are (x, t)."""
    g, p, w, _ = _streams(seed)
    nu = 0.01 / math.pi
    xs = np.linspace(-1.0, 1.0, n_strips + 1)
    n_res = max(1, int(round(5000 * scale)))
    n_ic = max(1, int(round(256 * scale)))
    n_bc = max(1, int(round(100 * scale)))
    n_i = max(1, int(round(200 * scale)))
    subs = []
    for q in range(n_strips):
        widths = [2] + [50] * 6 + [1]
        x0, x1 = xs[q], xs[q + 1]
        res = _box_points(p, n_res, x0, x1, 0.0, 1.0)
        ic = np.stack([p.uniform(x0, x1, n_ic), np.zeros(n_ic)], 1)
        parts = [ic]
        targets = [-np.sin(np.pi * ic[:, 0])]
        if q == 0:
            bc = np.stack([np.full(n_bc, -1.0), p.uniform(0.0, 1.0, n_bc)], 1)
            parts.append(bc)
            targets.append(np.zeros(n_bc))
        if q == n_strips - 1:
            bc = np.stack([np.full(n_bc, 1.0), p.uniform(0.0, 1.0, n_bc)], 1)
            parts.append(bc)
            targets.append(np.zeros(n_bc))
        bnd = np.concatenate(parts, 0)
        gv = np.concatenate(targets, 0)[:, None]
        subs.append(Subdomain(widths=widths, loss_w=(1.0, 1.0, 1.0, 1.0), lr=1e-3,
                              res_xy=_f32(res), res_f=_f32(np.zeros((n_res, 1))),
                              bnd_xy=_f32(bnd), bnd_g=_f32(gv),
                              params=glorot_params(w, widths)))
    ifaces = []
    for q in range(n_strips - 1):
        pts = np.stack([np.full(n_i, xs[q + 1]), p.uniform(0.0, 1.0, n_i)], 1)
        ifaces.append(Interface(q, q + 1, _f32(pts), _f32([1.0, 0.0])))
    # evaluation grid 256 x 101 in (x, t); owners from the strips
    gx = np.linspace(-1.0, 1.0, 256)
    gt = np.linspace(0.0, 1.0, 101)
    X, T = np.meshgrid(gx, gt, indexing="ij")
    exy32 = _f32(np.stack([X.ravel(), T.ravel()], 1))
    ex = exy32.astype(np.float64)
    owner = -np.ones((len(ex), 4), np.int32)
    cnt = np.zeros(len(ex), np.int32)
    for q in range(n_strips):
        idx = np.nonzero((ex[:, 0] >= xs[q]) & (ex[:, 0] <= xs[q + 1]))[0]
        owner[idx, cnt[idx]] = q
        cnt[idx] += 1
    exact = burgers_exact(ex[:, 0], ex[:, 1], nu)[:, None]
    return Problem(name="c3_cpinn_burgers", method=METHOD_CPINN, pde=PDE_BURGERS1D,
                   coef=(nu,), subdomains=subs, interfaces=ifaces, eval_xy=exy32,
                   eval_owner=owner, eval_exact=exact)


def burgers_exact(x, t, nu, n_nodes=120):
    """Reference solution of the viscous Burgers problem with u0 = -sin(pi x)
    through the Cole-Hopf representation, evaluated by Gauss-Hermite
    quadrature (only used for the reported relative L2 error)."""
    x = np.asarray(x, float)
    t = np.asarray(t, float)
    out = np.empty_like(x)
    z, wq = np.polynomial.hermite.hermgauss(n_nodes)
    t0 = t <= 0
    out[t0] = -np.sin(np.pi * x[t0])
    xx = x[~t0][:, None]
    tt = t[~t0][:, None]
    s = np.sqrt(4.0 * nu * tt)
    y = xx - s * z[None, :]
    # phi(y) = exp(-cos(pi y) / (2 pi nu)); shift the exponent for stability
    expo = -np.cos(np.pi * y) / (2 * np.pi * nu)
    m = expo.max(axis=1, keepdims=True)
    e = np.exp(expo - m) * wq[None, :]
    num = (np.sin(np.pi * y) * e).sum(1)
    den = e.sum(1)
    out[~t0] = -num / den
    return out


def ns_cpinn_kovasznay(seed=0, scale=1.0, re=40.0):
    """The C4 problem with cPINN interfaces (Table 1 fluxes)."""
    return c4_xpinn_kovasznay(seed=seed, scale=scale, re=re, method=METHOD_CPINN)


def burgers_space_time(method, nx, nt, seed=0, scale=1.0, n_res=80000, width=20, depth=5,
                       n_ic=256, n_bc=100, n_iface=20, lr=8e-4):
    """The viscous Burgers problem of Sec. 7.5 (Eq. BE1: x in [-1,1], t in
    [0,1], nu = 0.01/pi, u(0,x) = -sin(pi x), u(t,+-1) = 0) on an nx x nt grid
    of space-time boxes, subdomain q = it * nx + ix.  Every subdomain has a
    2-20x5-1 tanh network and learning rate 8e-4; the 80k residual points of
    the whole domain are split evenly over the subdomains, and every common
    edge carries 20 interface points (Sec. 7.5).  Space interfaces x = const
    have normal (1, 0), time interfaces t = const normal (0, 1).  The 256
    initial points are split evenly over the first time slab and the 100
    points of each end line x = -1, +1 evenly over the time slabs.  Table 3
    pairs cPINN with nt = 1 and XPINN with nt > 1; the flux of the cPINN
    form is the space-time flux (u^2/2 - nu u_x, u), so a cPINN time
    interface is defined as well.  method="hybrid" is the combination the
    conclusions propose: cPINN flux matching across space interfaces, XPINN
    residual continuity across time interfaces.  Inputs are (x, t)."""
    if nx < 1 or nt < 1:
        raise ValueError("nx and nt must be positive")
    if method not in (METHOD_CPINN, METHOD_XPINN, "hybrid"):
        raise ValueError(f"unknown method {method}")
    hybrid = method == "hybrid"
    g, p, w, _ = _streams(seed)
    nu = 0.01 / math.pi
    xs = np.linspace(-1.0, 1.0, nx + 1)
    ts = np.linspace(0.0, 1.0, nt + 1)
    per = lambda total, parts: max(1, int(round(total * scale / parts)))
    n_r, n_0, n_b, n_i = per(n_res, nx * nt), per(n_ic, nx), per(n_bc, nt), per(n_iface, 1)
    widths = [2] + [width] * depth + [1]
    subs = []
    for it in range(nt):
        for ix in range(nx):
            x0, x1, t0, t1 = xs[ix], xs[ix + 1], ts[it], ts[it + 1]
            res = _box_points(p, n_r, x0, x1, t0, t1)
            parts, targets = [np.zeros((0, 2))], [np.zeros(0)]
            if it == 0:
                ic = np.stack([p.uniform(x0, x1, n_0), np.zeros(n_0)], 1)
                parts.append(ic)
                targets.append(-np.sin(np.pi * ic[:, 0]))
            for edge, on in ((-1.0, ix == 0), (1.0, ix == nx - 1)):
                if on:
                    parts.append(np.stack([np.full(n_b, edge), p.uniform(t0, t1, n_b)], 1))
                    targets.append(np.zeros(n_b))
            bnd = np.concatenate(parts, 0)
            gv = np.concatenate(targets, 0)[:, None]
            subs.append(Subdomain(widths=list(widths), loss_w=(1.0, 1.0, 1.0, 1.0), lr=lr,
                                  res_xy=_f32(res), res_f=_f32(np.zeros((n_r, 1))),
                                  bnd_xy=_f32(bnd), bnd_g=_f32(gv),
                                  params=glorot_params(w, widths)))
    ifaces = []
    for it in range(nt):
        for ix in range(nx):
            q = it * nx + ix
            if ix + 1 < nx:   # space interface x = xs[ix+1], open in t
                pts = _segment_points(p, n_i, (xs[ix + 1], ts[it]), (xs[ix + 1], ts[it + 1]))
                ifaces.append(Interface(q, q + 1, _f32(pts), _f32([1.0, 0.0]),
                                        METHOD_CPINN if hybrid else None))
            if it + 1 < nt:   # time interface t = ts[it+1], open in x
                pts = _segment_points(p, n_i, (xs[ix], ts[it + 1]), (xs[ix + 1], ts[it + 1]))
                ifaces.append(Interface(q, q + nx, _f32(pts), _f32([0.0, 1.0]),
                                        METHOD_XPINN if hybrid else None))
    gx = np.linspace(-1.0, 1.0, 256)
    gt = np.linspace(0.0, 1.0, 101)
    X, T = np.meshgrid(gx, gt, indexing="ij")
    exy32 = _f32(np.stack([X.ravel(), T.ravel()], 1))
    ex = exy32.astype(np.float64)
    owner = -np.ones((len(ex), 4), np.int32)
    cnt = np.zeros(len(ex), np.int32)
    for it in range(nt):
        for ix in range(nx):
            inside = ((ex[:, 0] >= xs[ix]) & (ex[:, 0] <= xs[ix + 1]) &
                      (ex[:, 1] >= ts[it]) & (ex[:, 1] <= ts[it + 1]))
            idx = np.nonzero(inside)[0]
            owner[idx, cnt[idx]] = it * nx + ix
            cnt[idx] += 1
    exact = burgers_exact(ex[:, 0], ex[:, 1], nu)[:, None]
    name = f"burgers_{method}_{nx}x{nt}"
    return Problem(name=name, method=METHOD_CPINN if hybrid else method, pde=PDE_BURGERS1D, coef=(nu,), subdomains=subs,
                   interfaces=ifaces, eval_xy=exy32, eval_owner=owner, eval_exact=exact,
                   meta={"nx": nx, "nt": nt})


def c4_xpinn_kovasznay(seed=0, scale=1.0, re=40.0, method=METHOD_XPINN):
    """XPINN, steady NS (Eq. NSEq) at Re = 40 with the Kovasznay closed form on
    [-0.5,1] x [-0.5,1.5], 3x3 subdomains, nets 2-60x5-3, 10k residual points
    each, 100 exact (u,v,p) points per outer segment, 200 per interface.
    method="cpinn" matches the momentum and mass fluxes of Table 1 across the
    interfaces instead of the residuals."""
    g, p, w, _ = _streams(seed)
    n_res = max(1, int(round(10000 * scale)))
    n_b = max(1, int(round(100 * scale)))
    n_i = max(1, int(round(200 * scale)))
    name = "c4_xpinn_kovasznay" if method == METHOD_XPINN else "ns_cpinn_kovasznay"
    return _box_grid_problem(
        name, method, PDE_NS2D, (re,), g, p, w,
        [-0.5, 0.0, 0.5, 1.0], [-0.5, 1.0 / 6.0, 5.0 / 6.0, 1.5],
        lambda r, q: [2] + [60] * 5 + [3], lambda r, q: n_res, n_b, n_i,
        lambda x, y: kovasznay_exact(x, y, re), lambda x, y: np.zeros((len(x), 3)),
        (1.0, 1.0, 1.0, 1.0), 1e-3, (151, 201))


def star_radius(theta, amp, phase, r0=0.3):
    """r(theta) = r0 (1 + sum_{k=2..5} amp_k cos(k theta + phase_k))."""
    r = np.ones_like(theta)
    for i, k in enumerate(range(2, 6)):
        r = r + amp[i] * np.cos(k * theta + phase[i])
    return r0 * r


def _in_star(xy, center, amp, phase):
    d = xy - center[None, :]
    return np.hypot(d[:, 0], d[:, 1]) < star_radius(np.arctan2(d[:, 1], d[:, 0]), amp, phase)


def _nearest(xy, sites):
    d2 = ((xy[:, None, :] - sites[None, :, :]) ** 2).sum(-1)
    return np.argmin(d2, 1), d2


#: per-subdomain activations and residual counts of Table 4 (10 subdomains)
TABLE4_ACTS = ("tanh", "sin", "cos", "tanh", "sin", "cos", "tanh", "sin", "cos", "tanh")
TABLE4_NRES = (3000, 4000, 5000, 4000, 3000, 4000, 800, 3000, 5000, 4000)


def c5_xpinn_inverse_diffusion(seed=0, scale=1.0, n_cells=10, table4=False):
    """XPINN for the inverse steady diffusion problem div(K grad u) = f
    (Eq. heq, Sec. 7.6): the conductivity K is a second network per subdomain,
    known only on the outer boundary, while u is observed inside the domain.

    Stands in for the US-map geometry: a seeded star-shaped domain
    r(theta) = 0.3 (1 + sum_{k=2..5} a_k cos(k theta + phi_k)) around (0.5, 0.5),
    a_k ~ U[-0.06, 0.06], cut into n_cells Voronoi cells (sites at least 0.08
    apart).  Per cell: u-net and K-net widths from {20,40,60,80,100} and
    3..6 hidden layers, drawn independently; U_int[1000,30000] residual
    points.  200 points on each shared Voronoi edge; 500 interior
    observations u + 1% noise; 400 outer-boundary points with u and K targets.
    Fields: u = sin(pi x) sin(pi y), K = 1 + 0.5 sin(2 pi x) cos(2 pi y).
    Subdomain.params holds [u-net | K-net] (canonical layout each).

    table4=True takes the network set-up of Table 4 instead: 3 hidden layers
    of 80 for both networks, the table's residual counts and per-subdomain
    activation (tanh, sin, cos in turn) with trainable slopes (n = 10)."""
    if table4 and n_cells != len(TABLE4_ACTS):
        raise ValueError("Table 4 lists 10 subdomains")
    g, p, w, nz = _streams(seed)
    center = np.array([0.5, 0.5])
    amp = g.uniform(-0.06, 0.06, 4)
    phase = g.uniform(0.0, 2 * np.pi, 4)
    rmax = 0.3 * (1 + 4 * 0.06)
    lo, hi = center - rmax, center + rmax

    def uniform_in_star(rng, n):
        out = np.zeros((0, 2))
        while out.shape[0] < n:
            c = rng.uniform(lo, hi, (max(64, 2 * (n - out.shape[0])), 2))
            out = np.concatenate([out, c[_in_star(c, center, amp, phase)]], 0)
        return out[:n]

    sites = np.zeros((0, 2))
    while sites.shape[0] < n_cells:
        c = uniform_in_star(g, 1)
        if sites.shape[0] == 0 or np.min(np.hypot(*(sites - c).T)) >= 0.08:
            sites = np.concatenate([sites, c], 0)
    wch = [20, 40, 60, 80, 100]
    uw, kw, nres = [], [], []
    for q in range(n_cells):
        uw.append([2] + [int(g.choice(wch))] * int(g.integers(3, 7)) + [1])
        kw.append([2] + [int(g.choice(wch))] * int(g.integers(3, 7)) + [1])
        nres.append(max(1, int(round(int(g.integers(1000, 30001)) * scale))))
    if table4:
        uw = kw = [[2, 80, 80, 80, 1]] * n_cells
        nres = [max(1, int(round(n * scale))) for n in TABLE4_NRES]

    # residual points: uniform in the star, kept by nearest site up to each quota
    res = [np.zeros((0, 2)) for _ in range(n_cells)]
    while any(res[q].shape[0] < nres[q] for q in range(n_cells)):
        c = uniform_in_star(p, 20000)
        own, _ = _nearest(c, sites)
        for q in range(n_cells):
            need = nres[q] - res[q].shape[0]
            if need > 0:
                res[q] = np.concatenate([res[q], c[own == q][:need]], 0)

    # interfaces: pieces of the bisector of two sites that are closer to them
    # than to any other site and inside the domain
    n_i = max(1, int(round(200 * scale)))
    tg = np.linspace(-1.0, 1.0, 20001)
    ifaces = []
    for a in range(n_cells):
        for b in range(a + 1, n_cells):
            m = 0.5 * (sites[a] + sites[b])
            nrm = (sites[b] - sites[a]) / np.linalg.norm(sites[b] - sites[a])
            d = np.array([-nrm[1], nrm[0]])

            def valid(t):
                pts = m[None, :] + t[:, None] * d[None, :]
                own, d2 = _nearest(pts, sites)
                da = d2[:, a]
                others = np.delete(d2, [a, b], axis=1)
                ok = _in_star(pts, center, amp, phase)
                if others.shape[1]:
                    ok &= (others > da[:, None]).all(1)
                return ok, pts

            ok, _ = valid(tg)
            if ok.sum() < 50:          # no shared edge (or a sliver) inside the domain
                continue
            t_lo, t_hi = tg[ok].min(), tg[ok].max()
            got = np.zeros((0, 2))
            while got.shape[0] < n_i:
                t = p.uniform(t_lo, t_hi, 2 * n_i)
                okt, pts = valid(t)
                got = np.concatenate([got, pts[okt]], 0)
            ifaces.append(Interface(a, b, _f32(got[:n_i]), _f32(nrm)))

    # data: interior observations of u with 1% noise, boundary u and K
    n_obs = max(1, int(round(500 * scale)))
    n_bd = max(1, int(round(400 * scale)))
    obs = uniform_in_star(p, n_obs)
    u_obs, _, _ = diffusion_fields(obs[:, 0], obs[:, 1])
    u_obs = u_obs + 0.01 * np.std(u_obs) * nz.standard_normal(n_obs)
    th = p.uniform(0.0, 2 * np.pi, n_bd)
    rb = star_radius(th, amp, phase)
    bd = center[None, :] + rb[:, None] * np.stack([np.cos(th), np.sin(th)], 1)
    u_bd, k_bd, _ = diffusion_fields(bd[:, 0], bd[:, 1])
    own_obs, _ = _nearest(obs, sites)
    own_bd, _ = _nearest(bd, sites)

    subs = []
    for q in range(n_cells):
        r = res[q]
        _, _, f = diffusion_fields(r[:, 0], r[:, 1])
        so, sb = own_obs == q, own_bd == q
        dxy = np.concatenate([obs[so], bd[sb]], 0)
        dg = np.concatenate([u_obs[so], u_bd[sb]], 0)[:, None]
        pu, pk = glorot_params(w, uw[q], table4), glorot_params(w, kw[q], table4)
        subs.append(Subdomain(widths=list(uw[q]), loss_w=(1.0, 1.0, 1.0, 1.0), lr=6e-3,
                              res_xy=_f32(r), res_f=_f32(f[:, None]), bnd_xy=_f32(dxy), bnd_g=_f32(dg),
                              params=np.concatenate([pu, pk]), aux_widths=list(kw[q]),
                              aux_xy=_f32(bd[sb]), aux_g=_f32(k_bd[sb][:, None]),
                              act=TABLE4_ACTS[q] if table4 else "tanh", adaptive=table4))
    # evaluation grid inside the star; owners = nearest site(s)
    gx = np.linspace(lo[0], hi[0], 201)
    X, Y = np.meshgrid(gx, np.linspace(lo[1], hi[1], 201), indexing="ij")
    exy = np.stack([X.ravel(), Y.ravel()], 1)
    exy = _f32(exy[_in_star(exy, center, amp, phase)])
    ex = exy.astype(np.float64)
    _, d2 = _nearest(ex, sites)
    dmin = d2.min(1, keepdims=True)
    tie = d2 <= dmin * (1 + 1e-9)
    owner = -np.ones((len(ex), 4), np.int32)
    for i in range(len(ex)):
        qs = np.nonzero(tie[i])[0][:4]
        owner[i, :len(qs)] = qs
    ue, ke, _ = diffusion_fields(ex[:, 0], ex[:, 1])
    return Problem(name="c5_table4_adaptive" if table4 else "c5_xpinn_inverse_diffusion", method=METHOD_XPINN,
                   pde=PDE_DIFFUSION2D_INV,
                   coef=(), subdomains=subs, interfaces=ifaces, eval_xy=exy, eval_owner=owner,
                   eval_exact=np.stack([ue, ke], 1),
                   meta={"sites": sites, "center": center, "amp": amp, "phase": phase})


WORKLOADS = {
    "c1_cpinn_poisson": c1_cpinn_poisson,
    "c2_xpinn_poisson": c2_xpinn_poisson,
    "c3_cpinn_burgers": c3_cpinn_burgers,
    "c4_xpinn_kovasznay": c4_xpinn_kovasznay,
    "c5_xpinn_inverse_diffusion": c5_xpinn_inverse_diffusion,
}

#: the space-time Burgers partitions of Table 3 (cPINN in space only, XPINN in
#: space and time), 80k residual points in every case
TABLE3_PARTITIONS = (("cpinn", 4, 1), ("cpinn", 8, 1), ("cpinn", 16, 1), ("cpinn", 32, 1),
                     ("xpinn", 2, 2), ("xpinn", 4, 2), ("xpinn", 4, 4), ("xpinn", 8, 4))


def _table3_entry(method, nx, nt):
    def make(seed=0, scale=1.0):
        return burgers_space_time(method, nx, nt, seed=seed, scale=scale)
    make.__name__ = f"burgers_st_{method}_{nx}x{nt}"
    return make


for _m, _nx, _nt in TABLE3_PARTITIONS + (("hybrid", 4, 4),):
    WORKLOADS[f"burgers_st_{_m}_{_nx}x{_nt}"] = _table3_entry(_m, _nx, _nt)
WORKLOADS["ns_cpinn_kovasznay"] = ns_cpinn_kovasznay


def c5_table4_adaptive(seed=0, scale=1.0):
    """The inverse problem with the networks of Table 4 (adaptive tanh / sin /
    cos per subdomain, 3 x 80)."""
    return c5_xpinn_inverse_diffusion(seed=seed, scale=scale, table4=True)


WORKLOADS["c5_table4_adaptive"] = c5_table4_adaptive


def make_problem(name, seed=0, scale=1.0, **kw):
    return WORKLOADS[name](seed=seed, scale=scale, **kw)


def custom_box_problem(method, pde, nx, ny, widths_list, n_res_list, n_bnd_seg, n_iface,
                       seed=0, coef=(), loss_w=(1.0, 1.0, 1.0, 1.0), lr=1e-3,
                       domain=(0.0, 1.0, 0.0, 1.0)):
    """Small custom Cartesian problems for tests (ragged counts, mixed widths)."""
    g, p, w, _ = _streams(seed)
    xs = list(np.linspace(domain[0], domain[1], nx + 1))
    ys = list(np.linspace(domain[2], domain[3], ny + 1))
    if pde == PDE_POISSON2D:
        ex, fo = poisson_exact, poisson_forcing
    elif pde == PDE_NS2D:
        re = coef[0]
        ex = lambda x, y: kovasznay_exact(x, y, re)
        fo = lambda x, y: np.zeros((len(x), 3))
    elif pde == PDE_BURGERS1D:
        ex = lambda x, y: -np.sin(np.pi * x) * (y == 0)
        fo = lambda x, y: np.zeros(len(x))
    else:
        raise ValueError(pde)
    return _box_grid_problem("custom", method, pde, coef, g, p, w, xs, ys,
                             lambda r, q: list(widths_list[q]), lambda r, q: int(n_res_list[q]),
                             n_bnd_seg, n_iface, ex, fo, loss_w, lr, (21, 21))


def with_activations(prob, acts, adaptive=True, slope_n=10.0):
    """Give subdomain q the activation acts[q % len(acts)] and, if adaptive,
    trainable slopes initialised to n a^k = 1 (appended after the layers of each
    of its networks).  Modifies and returns prob."""
    for q, sd in enumerate(prob.subdomains):
        sd.act = acts[q % len(acts)]
        if adaptive and not sd.adaptive:
            nu = param_count(sd.widths)
            parts = [sd.params[:nu], np.full(len(sd.widths) - 2, 1.0 / slope_n)]
            if sd.aux_widths is not None:
                parts += [sd.params[nu:], np.full(len(sd.aux_widths) - 2, 1.0 / slope_n)]
            sd.params = np.concatenate(parts).astype(np.float32)
            sd.adaptive, sd.slope_n = True, slope_n
    return prob
