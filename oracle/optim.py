"""AdamW (Loshchilov & Hutter, "Decoupled weight decay regularization", ICLR 2019), FP64,
as used for training in Sec. 6.3 (betas (0.8, 0.985), weight decay 0.02):
    m = b1 m + (1 - b1) g;   v = b2 v + (1 - b2) g^2
    p = p - lr * (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd * p)
"""
import numpy as np


def adamw_step(p, g, m, v, t, lr, b1=0.8, b2=0.985, eps=1e-8, wd=0.02):
    p, g, m, v = (np.asarray(a, dtype=np.float64) for a in (p, g, m, v))
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v
