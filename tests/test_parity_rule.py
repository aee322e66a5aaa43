"""CPU checks of the GPU parity rule itself (tests/parity_util.py): a gradient
within rounding of the oracle's passes, and one wrong entry of a layer, too
small for the 2-norm bars, fails the element-wise bar."""
import numpy as np
import pytest

import oracle
import parity_util as P
from paper_2104_10013_amd import workloads as W


@pytest.fixture(scope="module")
def ref():
    prob = W.custom_box_problem("xpinn", "poisson2d", 2, 1, [[2, 40, 40, 40, 1]] * 2, [300, 250],
                                n_bnd_seg=20, n_iface=30, seed=4)
    params = [s.params for s in prob.subdomains]
    terms, grads = oracle.loss_and_grad(prob, params)
    return prob, params, terms, grads


def test_rounding_level_differences_pass(ref):
    prob, params, terms, grads = ref
    rng = np.random.default_rng(0)
    g = [r * (1 + 2e-7 * rng.standard_normal(r.size)) for r in grads]
    P.compare(prob, params, terms.astype(np.float32), g, ref=(terms, grads))


def test_one_wrong_entry_fails_the_element_bar_only(ref):
    prob, params, terms, grads = ref
    g = [r.copy() for r in grads]
    sd = prob.subdomains[0]
    grp = P.layer_groups(sd.widths)
    idx = grp[2]                         # second hidden layer: W^3 (40 x 40) and b^3
    r = grads[0][idx]
    i = idx[int(np.argmin(np.abs(np.abs(r) - np.sqrt(np.mean(r * r)))))]   # an entry of typical size
    g[0][i] *= 1 + 2e-4
    # the 2-norm bars do not see it ...
    assert np.linalg.norm(g[0] - grads[0]) / np.linalg.norm(grads[0]) < P.GRAD_RTOL
    assert np.linalg.norm(g[0][idx] - grads[0][idx]) / np.linalg.norm(grads[0][idx]) < P.GRAD_RTOL
    # ... the element bar does
    with pytest.raises(AssertionError, match="element ratio"):
        P.compare(prob, params, terms.astype(np.float32), g, ref=(terms, grads))


def test_groups_cover_every_parameter_once(ref):
    prob = ref[0]
    for s in prob.subdomains:
        idx = np.concatenate(P.layer_groups(s.widths, s.aux_widths, s.adaptive))
        assert np.array_equal(np.sort(idx), np.arange(W.param_count(s.widths, s.adaptive)))
    p5 = W.c5_table4_adaptive(seed=0, scale=0.02)
    s = p5.subdomains[0]
    idx = np.concatenate(P.layer_groups(s.widths, s.aux_widths, s.adaptive))
    n = W.param_count(s.widths, s.adaptive) + W.param_count(s.aux_widths, s.adaptive)
    assert np.array_equal(np.sort(idx), np.arange(n))
