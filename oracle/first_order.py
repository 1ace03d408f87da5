"""First-order baseline on the same gradients (test infrastructure).

The local-Newton sweep is compared against plain gradient descent and Adam
driven by the very gradients its blocks carry (the paper's claims of fewer
iterations than first-order training, Sec. 1 and Sec. 5, are measured against
this).  Written in plain NumPy from the definitions:

* the gradient of each kernel with respect to position, the left rotation
  vector omega (q <- exp(omega/2) q), the linear scale, the opacity and the SH
  coefficients; the SH gradient of channel ch is sum over views of
  gamma_{v,ch} Y(r_v) (the colour of the splat is Y(r_v)^T c_ch, Sec. 4.2
  colour paragraph);
* gradient descent: x <- x - lr g;
* Adam (Kingma and Ba, 2015): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
  x <- x - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps);
* the parameter updates of the Newton apply: rotation by the exponential map
  of the step in omega, scale kept >= scale_floor * s, opacity kept in
  [opac_eps, 1 - opac_eps].

Only kernels the primary view sees are updated (their moments too), as in the
Newton sweep.  Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``
may import this module.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O

GROUPS = ("position", "rotation", "scaling", "opacity", "colour")


def n_features(K: int) -> int:
    """Gradient entries per kernel: position 3, omega 3, scale 3, opacity 1, colour 3K."""
    return 10 + 3 * K


def gradient(summed, V, K):
    """Per-kernel gradient [n][10 + 3K] from the summed blocks (solve layout [n][39 + 10V])."""
    S = np.asarray(summed, np.float64)
    n = S.shape[0]
    out = np.zeros((n, n_features(K)))
    out[:, 0:3] = S[:, 0:3]
    out[:, 3:6] = S[:, 12:15]
    out[:, 6:9] = S[:, 24:27]
    out[:, 9] = S[:, 36]
    for k in range(n):
        for v in range(V):
            b = O.NB_BASE + O.NB_VIEW * v
            if not S[k, b + 9] > 0.0:  # the view does not see the kernel
                continue
            Y = O.sh_basis(K, S[k, b + 6:b + 9])
            for ch in range(3):
                out[k, 10 + ch * K:10 + (ch + 1) * K] += S[k, b + ch] * Y
    return out


def _qexp(w):
    th = float(np.linalg.norm(w))
    if th == 0.0:
        return np.array([1.0, 0.0, 0.0, 0.0])
    return np.concatenate([[np.cos(0.5 * th)], np.sin(0.5 * th) * w / th])


def _qmul(a, b):
    return np.array([a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3],
                     a[0] * b[1] + a[1] * b[0] + a[2] * b[3] - a[3] * b[2],
                     a[0] * b[2] + a[2] * b[0] + a[3] * b[1] - a[1] * b[3],
                     a[0] * b[3] + a[3] * b[0] + a[1] * b[2] - a[2] * b[1]])


def step(g, summed, V, lr, adam=True, state=None, t=1, beta1=0.9, beta2=0.999, eps=1e-15,
         scale_floor=0.1, opac_eps=1e-6, mask=31):
    """One first-order step.  lr: five learning rates (position, rotation, scaling, opacity,
    colour).  state: (m, v) arrays [n][10 + 3K] (Adam; updated in place), t the step count.
    Returns the new kernels (float64)."""
    out = O.G64.of(g).copy()
    K = out.K
    grad = gradient(summed, V, K)
    S = np.asarray(summed, np.float64)
    seen = S[:, 38] > 0.0
    slices = [slice(0, 3), slice(3, 6), slice(6, 9), slice(9, 10), slice(10, 10 + 3 * K)]
    upd = np.zeros_like(grad)
    for gi, sl in enumerate(slices):
        if not mask & (1 << gi):
            continue
        gg = grad[:, sl]
        if adam:
            m, v = state
            m[seen, sl] = beta1 * m[seen, sl] + (1.0 - beta1) * gg[seen]
            v[seen, sl] = beta2 * v[seen, sl] + (1.0 - beta2) * gg[seen] ** 2
            mh = m[:, sl] / (1.0 - beta1 ** t)
            vh = v[:, sl] / (1.0 - beta2 ** t)
            upd[:, sl] = lr[gi] * mh / (np.sqrt(vh) + eps)
        else:
            upd[:, sl] = lr[gi] * gg
    for k in np.nonzero(seen)[0]:
        if mask & 1:
            out.pos[:, k] -= upd[k, 0:3]
        if mask & 2:
            q = _qmul(_qexp(-upd[k, 3:6]), out.rot[:, k])
            out.rot[:, k] = q / np.linalg.norm(q)
        if mask & 4:
            s = out.scale[:, k]
            out.scale[:, k] = np.maximum(s - upd[k, 6:9], scale_floor * s)
        if mask & 8:
            out.opac[k] = min(max(out.opac[k] - upd[k, 9], opac_eps), 1.0 - opac_eps)
        if mask & 16:
            out.sh[:, :, k] -= upd[k, 10:10 + 3 * K].reshape(3, K)
    return out
