"""Adam update (oracle, FP64).  Test infrastructure only.

The paper trains with Adam (Sec. III-G, Sec. IV-B: learning rate 0.01); the
remaining hyper-parameters are not stated, so the usual defaults
beta1 = 0.9, beta2 = 0.999, eps = 1e-8 are taken.  Step t counts from 1.
"""
import numpy as np


def adam_step(param, grad, m, v, t, lr=0.01, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step on float64 numpy arrays; returns (param, m, v)."""
    param = np.asarray(param, np.float64)
    grad = np.asarray(grad, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * grad
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * grad * grad
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return param - lr * m_hat / (np.sqrt(v_hat) + eps), m, v
