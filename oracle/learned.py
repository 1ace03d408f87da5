"""FP64 oracle of the learned per-kernel step scale (test infrastructure only).

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may use this module.

The paper's overshoot control (Sec. 4.3, eq. tildel) adds the Hessians and
gradients of the |N_t| nearest training views to those of the primary view, so
that the local Newton step of a kernel does not overshoot what the neighbouring
views see.  The learned form replaces those extra views on most sweeps by a small
network that predicts, per kernel and attribute group, how much of the
primary-only step the full rule would keep:

* label (from a sweep that runs the full rule): for group y,
  alpha_eff = <Delta_aug, Delta_prim> / |Delta_prim|^2, clipped to [0, 1.5]: the
  length of the full-rule step projected on the primary-only step, in units of
  the primary-only step;
* features: 16 per kernel from the primary view's blocks alone, and the residual the
  neighbouring views left at the kernel in its last full-rule sweep (``orc_features``,
  ``neighbour_residual``);
* network: 17 -> 32 (ReLU) -> 5, output 1.5 sigmoid, one scale per group
  (position, rotation, scaling, opacity, colour);
* training: mean squared error over the labelled (kernel, group) entries, Adam.

Parameter vector layout (741 values): W1 [32][17] row-major, b1 [32],
W2 [5][32] row-major, b2 [5].
"""
from __future__ import annotations

import ctypes

import numpy as np

from oracle import oracle as O

N_IN, N_HID, N_OUT = 17, 32, 5
N_PARAMS = N_HID * N_IN + N_HID + N_OUT * N_HID + N_OUT
ALPHA_MAX = 1.5
# step-vector columns of each group (position 3, rotation angle 1, scaling 3, opacity 1, colour 3K)
GROUP_COLS = [slice(0, 3), slice(3, 4), slice(7, 10), slice(10, 11), None]
MIN_STEP_SQ = 1e-30


# feature status codes: not seen by the primary, features in range, seen but out of range
FEAT_HIDDEN, FEAT_OK, FEAT_OUT_OF_RANGE = 0, 1, 2


def features(g, cam, o, summed, V, resid=None):
    """Per-kernel features [n][17] and status codes [n] (FEAT_*) from the summed blocks and the
    cached neighbouring-view residuals resid [n] (None: 0)."""
    g64 = O.G64.of(g)
    feat = np.zeros((g64.n, N_IN))
    ok = np.zeros(g64.n, np.uint8)
    r = None if resid is None else np.ascontiguousarray(resid, np.float64)
    O.lib().orc_features(ctypes.c_int(g64.n), ctypes.c_int(g64.K), O._p(g64.pos), O._p(g64.rot),
                         O._p(g64.scale), O._p(g64.opac), O._p(O.cam_vec(cam)), O._p(o), ctypes.c_int(V),
                         O._p(np.ascontiguousarray(summed, np.float64)), O._p(r) if r is not None else None,
                         O._p(feat), O._p(ok))
    return feat, ok


def neighbour_residual(summed, V, prev):
    """The residual the neighbouring (secondary) views leave at each kernel, from the summed blocks
    of a full-rule sweep: for kernels the primary sees and some secondary view v >= 1 covers,
    sum over those views of |gamma_v| / (|gamma_0| + 1e-30) (gamma_v: the view's colour gradient);
    other kernels keep prev."""
    S = np.asarray(summed, np.float64)
    out = np.array(prev, np.float64, copy=True)
    base = O.NB_BASE

    def gnorm(v):
        return np.sqrt((S[:, base + O.NB_VIEW * v:base + O.NB_VIEW * v + 3] ** 2).sum(1))

    sec = np.zeros(S.shape[0])
    seen = np.zeros(S.shape[0], bool)
    for v in range(1, V):
        cov = S[:, base + O.NB_VIEW * v + 9] > 0
        sec[cov] += gnorm(v)[cov]
        seen |= cov
    upd = seen & (S[:, 38] > 0)
    out[upd] = sec[upd] / (gnorm(0)[upd] + 1e-30)
    return out


def unpack(params):
    p = np.asarray(params, np.float64)
    i = 0
    W1 = p[i:i + N_HID * N_IN].reshape(N_HID, N_IN)
    i += N_HID * N_IN
    b1 = p[i:i + N_HID]
    i += N_HID
    W2 = p[i:i + N_OUT * N_HID].reshape(N_OUT, N_HID)
    i += N_OUT * N_HID
    b2 = p[i:i + N_OUT]
    return W1, b1, W2, b2


def forward(params, F):
    """alpha [n][5] = 1.5 sigmoid(W2 relu(W1 f + b1) + b2) for each feature row f."""
    W1, b1, W2, b2 = unpack(params)
    z1 = np.asarray(F, np.float64) @ W1.T + b1
    h = np.maximum(z1, 0.0)
    z2 = h @ W2.T + b2
    return ALPHA_MAX / (1.0 + np.exp(-z2))


def loss_grad(params, F, label, mask):
    """Mean squared error over the masked (kernel, group) entries and its gradient [709],
    by the chain rule through the two layers."""
    W1, b1, W2, b2 = unpack(params)
    F = np.asarray(F, np.float64)
    mask = np.asarray(mask, np.float64)
    cnt = max(float(mask.sum()), 1.0)
    z1 = F @ W1.T + b1
    h = np.maximum(z1, 0.0)
    z2 = h @ W2.T + b2
    sg = 1.0 / (1.0 + np.exp(-z2))
    a = ALPHA_MAX * sg
    r = (a - label) * mask
    loss = float((r * r).sum() / cnt)
    d_a = 2.0 * r / cnt
    d_z2 = d_a * ALPHA_MAX * sg * (1.0 - sg)
    gW2 = d_z2.T @ h
    gb2 = d_z2.sum(0)
    d_h = d_z2 @ W2
    d_z1 = d_h * (z1 > 0.0)
    gW1 = d_z1.T @ F
    gb1 = d_z1.sum(0)
    return loss, np.concatenate([gW1.ravel(), gb1, gW2.ravel(), gb2])


def adam(params, m, v, t, grad, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1); returns new (params, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def labels(steps_prim, steps_aug, dec_prim, K, ok=None):
    """alpha_eff [n][5] and mask [n][5] from primary-only and full-rule steps [n][11 + 3K]; with the
    feature status codes ok, entries of kernels whose features were not in range are masked."""
    n = steps_prim.shape[0]
    lab = np.zeros((n, N_OUT))
    msk = np.zeros((n, N_OUT))
    vis = np.asarray(dec_prim)[:, 0] >= -1
    if ok is not None:
        vis = vis & (np.asarray(ok) == FEAT_OK)
    for gi, sl in enumerate(GROUP_COLS):
        sl = slice(11, 11 + 3 * K) if sl is None else sl
        p = np.asarray(steps_prim, np.float64)[:, sl]
        a = np.asarray(steps_aug, np.float64)[:, sl]
        pp = (p * p).sum(1)
        good = vis & (pp > MIN_STEP_SQ)
        lab[good, gi] = np.clip((a * p).sum(1)[good] / pp[good], 0.0, ALPHA_MAX)
        msk[good, gi] = 1.0
    return lab, msk


def label_error(alpha, lab, msk):
    """(sum of mask |alpha - label|, sum of mask): the network's error against the overshoot rule."""
    m = np.asarray(msk, np.float64)
    return float((np.abs(np.asarray(alpha, np.float64) - lab) * m).sum()), float(m.sum())
