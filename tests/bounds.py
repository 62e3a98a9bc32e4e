"""Error bounds used as test tolerances, derived from the arithmetic.

bf16_forward_bound: how far a forward pass of the learned-halo network can
move from the plain FP64 forward pass when every layer's inputs and weights
are rounded to BF16 (8 significant bits, unit roundoff u = 2^-9) and the dot
products are accumulated in FP32 (64 terms, at most 64 roundings of 2^-24
each).  Per layer, with exact activations x, weights W and an input error
e_in (elementwise, |x_hat - x| <= e_in):

    |r(x_hat) r(w) - x w| <= |w| |x_hat - x| (1 + u)^2 + |x_hat| |w| (2u + u^2)

summed over the inputs, plus the FP32 accumulation term
gamma |W| (|x| + e_in) (1 + u)^2 with gamma = 64 * 2^-24.  ReLU is
1-Lipschitz, so the bound of a layer's output is the next layer's e_in.
"""
import numpy as np

U_BF16 = 2.0 ** -9
GAMMA_F32 = 64 * 2.0 ** -24


def _layer(W, x, e_in):
    aW = np.abs(W)
    u = U_BF16
    mag = np.abs(x) + e_in
    return (e_in @ aW.T) * (1 + u) ** 2 + (mag @ aW.T) * (2 * u + u * u) + GAMMA_F32 * (mag @ aW.T) * (1 + u) ** 2


def bf16_forward_bound(theta, X):
    """Elementwise bound (n, 16) on |forward_bf16(X) - forward_fp64(X)|."""
    from oracle import mlp
    p = mlp.unpack(theta)
    X = np.asarray(X, dtype=np.float64)
    _, (X0, Z1, H1, Z2, H2) = mlp.forward(theta, X)
    e1 = _layer(p["W1"], X0, np.zeros_like(X0))
    e2 = _layer(p["W2"], H1, e1)
    e3 = _layer(p["W3"], H2, e2)
    return e3
