"""Small shared helpers for the test suite (no method arithmetic)."""
import numpy as np


def quad_weights3(w):
    """Tensor-product weights w_i w_j w_k in [k][j][i] order."""
    return w[None, None, :] * w[None, :, None] * w[:, None, None]


def rel_err_per_var(a, b):
    """max|a_v - b_v| / max|b_v| for each of the 5 state variables."""
    a = np.asarray(a)
    b = np.asarray(b)
    out = []
    for v in range(a.shape[0]):
        den = np.abs(b[v]).max()
        out.append(np.abs(a[v] - b[v]).max() / (den if den > 0 else 1.0))
    return np.array(out)
