"""Helpers shared by the GPU parity tests (comparison rules only)."""
import numpy as np

import oracle

# "1e-5 relative": each loss term within 1e-5 * max(|term|, 1e-3 * J_q); each
# subdomain gradient within 1e-5 * ||g_q|| in the 2-norm, also per layer tensor.
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


def compare(prob, params, lt_gpu, g_gpu, loss_rtol=LOSS_RTOL, grad_rtol=GRAD_RTOL, per_layer=True, ref=None):
    """Compare GPU loss terms / gradients with the FP64 oracle (or with ref =
    (terms, grads) it computed before); returns the worst relative errors
    (loss, grad) and raises AssertionError on failure."""
    terms, grads = ref if ref is not None else oracle.loss_and_grad(prob, params)
    lt = np.asarray(lt_gpu, np.float64)
    worst_l, worst_g = 0.0, 0.0
    for q in range(prob.n_sd):
        J = abs(terms[q, 0])
        for k in range(5):
            scale = max(abs(terms[q, k]), 1e-3 * J, 1e-30)
            err = abs(lt[q, k] - terms[q, k]) / scale
            worst_l = max(worst_l, err)
            assert err <= loss_rtol, f"sd {q} term {k}: gpu {lt[q, k]!r} oracle {terms[q, k]!r} rel {err:.3e}"
        g = np.asarray(g_gpu[q], np.float64)
        ref = grads[q]
        nref = np.linalg.norm(ref)
        err = np.linalg.norm(g - ref) / max(nref, 1e-30)
        worst_g = max(worst_g, err)
        assert err <= grad_rtol, f"sd {q} grad rel {err:.3e} (|g|={nref:.3e})"
        if per_layer:
            sd = prob.subdomains[q]
            for k, sl in enumerate(layer_slices(sd.widths, sd.aux_widths, getattr(sd, "adaptive", False))):
                r = ref[sl]
                nr = np.linalg.norm(r)
                if nr == 0.0 or nr < 1e-6 * nref:   # (a zero gradient is checked as a whole above)
                    continue
                e = np.linalg.norm(g[sl] - r) / nr
                assert e <= 10 * grad_rtol, f"sd {q} tensor {k} rel {e:.3e}"
    return worst_l, worst_g
