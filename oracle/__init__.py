"""FP64 CPU oracle: test infrastructure only (tests, smoke check, CPU baseline).

The product path never imports this package.
"""
from .pinn_oracle import (  # noqa: F401
    unpack, mlp, input_streams, residual, normal_flux, subdomain_terms, loss_and_grad,
    grad_of_total, adam_step, train, eval_stitched, rel_l2,
)
