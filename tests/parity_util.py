"""Helpers shared by the GPU parity tests (comparison rules only).

The bar is 1e-5 relative (FP32 kernels against the FP64 oracle):

* loss terms: each term within 1e-5 * max(|term|, 1e-3 * J_q);
* gradients, element by element, per layer: every entry g_i of layer k's
  weights W^k and bias b^k within 1e-5 * max(|r_i|, s_k) of the oracle's r_i,
  with the scale floor s_k = the root mean square of the oracle's entries of
  W^k and b^k together (an adaptive network's slopes form a group of their own
  with their own root mean square).  An FP32 gradient entry is a sum over
  points and streams, and its rounding error scales with the magnitudes of
  its terms, not with the sum: where the terms cancel (a bias entry whose
  per-point seeds change sign, e.g. the output bias fed by data misfits
  u - g and interface jumps) the relative error of the entry alone can exceed
  1e-5 at an absolute error of 1e-7.  The entries of W^k are sums of the same
  per-point seeds times activations of magnitude at most 1, so the layer's
  root mean square is a conservative stand-in for the term magnitudes of any
  of its entries; a one-entry output bias has no such scale of its own;
* gradients in the 2-norm, per layer (W^k with b^k; slopes) and per
  subdomain, each within 1e-5.

PARITY_LOG (environment) names a JSON-lines file that receives the worst
errors of every comparison (the figures quoted for each configuration).
"""
import json
import os

import numpy as np

import oracle

LOSS_RTOL = 1e-5
GRAD_RTOL = 1e-5


def layer_slices(widths, aux_widths=None, adaptive=False):
    """Slices of every weight matrix and bias vector (and of an adaptive
    network's slopes) in a subdomain's flat parameters (the u-network, then
    the K-network of the inverse problem)."""
    out, off = [], 0
    for wd in [widths] + ([aux_widths] if aux_widths is not None else []):
        for k in range(1, len(wd)):
            n = wd[k] * wd[k - 1]
            out.append(slice(off, off + n))
            off += n
            out.append(slice(off, off + wd[k]))
            off += wd[k]
        if adaptive:
            out.append(slice(off, off + len(wd) - 2))
            off += len(wd) - 2
    return out


def layer_groups(widths, aux_widths=None, adaptive=False):
    """Index groups of one subdomain's flat parameters for the element and
    2-norm checks: per network, each layer's weights and bias together, then
    an adaptive network's slopes."""
    sl = layer_slices(widths, aux_widths, adaptive)
    out, k = [], 0
    for wd in [widths] + ([aux_widths] if aux_widths is not None else []):
        for _ in range(1, len(wd)):
            out.append(np.r_[sl[k], sl[k + 1]])
            k += 2
        if adaptive:
            out.append(np.r_[sl[k]])
            k += 1
    return out


def grad_errors(g, ref, groups):
    """Worst element ratio |g_i - r_i| / max(|r_i|, s_k) and worst per-group
    2-norm error over the groups of one subdomain, and where they occur."""
    worst_e, where_e, worst_t, where_t = 0.0, None, 0.0, None
    for k, idx in enumerate(groups):
        r = ref[idx]
        if r.size == 0:
            continue
        d = np.abs(g[idx] - r)
        s_k = float(np.sqrt(np.mean(r * r)))
        if s_k == 0.0:
            # an all-zero reference group (e.g. a subdomain without points):
            # the GPU entries must be exactly zero as well
            e = float(d.max())
            if e > worst_e:
                worst_e, where_e = (np.inf if e > 0 else 0.0), (k, int(idx[int(d.argmax())]))
            continue
        ratio = d / np.maximum(np.abs(r), s_k)
        i = int(ratio.argmax())
        if ratio[i] > worst_e:
            worst_e, where_e = float(ratio[i]), (k, int(idx[i]))
        e = float(np.linalg.norm(g[idx] - r) / np.linalg.norm(r))
        if e > worst_t:
            worst_t, where_t = e, k
    return worst_e, where_e, worst_t, where_t


def compare(prob, params, lt_gpu, g_gpu, loss_rtol=LOSS_RTOL, grad_rtol=GRAD_RTOL, per_layer=True, ref=None,
            label=None):
    """Compare GPU loss terms / gradients with the FP64 oracle (or with ref =
    (terms, grads) it computed before); returns the worst relative errors
    (loss, grad in the 2-norm) and raises AssertionError on failure.
    per_layer=False skips the element and per-tensor checks (only for
    comparisons whose reference is itself a loose approximation)."""
    terms, grads = ref if ref is not None else oracle.loss_and_grad(prob, params)
    lt = np.asarray(lt_gpu, np.float64)
    worst_l, worst_g, worst_e, worst_t = 0.0, 0.0, 0.0, 0.0
    fails = []
    for q in range(prob.n_sd):
        J = abs(terms[q, 0])
        for k in range(5):
            scale = max(abs(terms[q, k]), 1e-3 * J, 1e-30)
            err = abs(lt[q, k] - terms[q, k]) / scale
            worst_l = max(worst_l, err)
            if err > loss_rtol:
                fails.append(f"sd {q} term {k}: gpu {lt[q, k]!r} oracle {terms[q, k]!r} rel {err:.3e}")
        g = np.asarray(g_gpu[q], np.float64)
        r = grads[q]
        nref = np.linalg.norm(r)
        if nref == 0.0:
            err = float(np.abs(g).max()) if g.size else 0.0
            if err != 0.0:
                fails.append(f"sd {q}: oracle gradient is zero, gpu max |g| {err:.3e}")
            continue
        err = np.linalg.norm(g - r) / nref
        worst_g = max(worst_g, err)
        if err > grad_rtol:
            fails.append(f"sd {q} grad rel {err:.3e} (|g|={nref:.3e})")
        if per_layer:
            sd = prob.subdomains[q]
            grp = layer_groups(sd.widths, sd.aux_widths, getattr(sd, "adaptive", False))
            e, we, t, wt = grad_errors(g, r, grp)
            worst_e, worst_t = max(worst_e, e), max(worst_t, t)
            if e > grad_rtol:
                k, i = we
                fails.append(f"sd {q} layer group {k} parameter {i}: gpu {g[i]!r} oracle {r[i]!r} "
                             f"element ratio {e:.3e}")
            if t > grad_rtol:
                fails.append(f"sd {q} layer group {wt} rel {t:.3e}")
    dump = os.environ.get("PARITY_DUMP")
    if dump and (fails or worst_e > 0.5 * grad_rtol):
        case = (label or os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0]).replace("/", "_").replace(":", "_")
        np.savez_compressed(os.path.join(dump, case + ".npz"),
                            **{f"g{q}": np.asarray(g_gpu[q], np.float64) for q in range(prob.n_sd)},
                            **{f"r{q}": np.asarray(grads[q], np.float64) for q in range(prob.n_sd)})
    log = os.environ.get("PARITY_LOG")
    if log:
        with open(log, "a") as f:
            f.write(json.dumps({"case": label or os.environ.get("PYTEST_CURRENT_TEST", "?").split(" ")[0],
                                "n_sd": int(prob.n_sd), "loss": worst_l, "grad_norm": worst_g,
                                "grad_layer": worst_t, "grad_element": worst_e, "ok": not fails}) + "\n")
    assert not fails, "; ".join(fails[:8])
    return worst_l, worst_g
