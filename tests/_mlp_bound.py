"""Per-element error bounds of the GPU's BF16 MLP against the FP64 oracle.

Both sides round the same operands to BF16 at the same points; they differ
only in how they form each value before it is rounded (FP32 accumulation on
the matrix cores against FP64 in the oracle).  Starting from the oracle's
own intermediate values, this carries an error radius e through the network
(the GPU's value lies within [v - e, v + e] of the oracle's v):

* a sum of n terms accumulated in FP32 in any order adds gamma(n) times the
  sum of the terms' magnitudes, gamma(n) = n u / (1 - n u), u = 2^-24;
* a BF16 rounding (round to nearest even, also behind a ReLU) is monotone,
  so the rounded GPU value lies between the roundings of v - e and v + e:
  the radius after rounding is 0 when both round to the oracle's value (no
  BF16 rounding boundary within the interval), else the larger gap;
* a ReLU mask (z > 0) is uncertain only when [z - e, z + e] straddles 0;
  there the masked value may be 0 or the unmasked one.

Nothing here uses a GPU value: the radii depend on the oracle's values and
on the operation counts alone.  Where no rounding boundary falls inside an
interval (almost everywhere), the bound is the FP32 accumulation error only,
so a rounding the GPU dropped or moved shows up as a violation.
"""
import numpy as np

from oracle import surrogate as S

U = 2.0 ** -24


def gamma(n):
    return n * U / (1.0 - n * U)


def _rounded(v, e, relu):
    f = (lambda a: S.bf16(np.maximum(a, 0.0))) if relu else S.bf16
    r = f(v)
    lo, hi = f(v - e), f(v + e)
    return np.maximum(r - lo, hi - r)


def _mask_err(z, ez, val, eval_):
    """Radius of val * [z > 0] given radii ez of z and eval_ of val."""
    pos = z - ez > 0
    neg = z + ez <= 0
    unc = ~(pos | neg)
    return np.where(pos, eval_, 0.0) + np.where(unc, np.abs(val) + eval_, 0.0)


def forward_bound(params, X):
    """(prediction [N], radius [N], state for backward_bound)."""
    out, cache = S.mlp_forward(params, X)
    Xb, Z1, H1, Z2, H2, W1, W2, W3 = cache
    p = S.unpack(np.asarray(params, np.float64))
    b1, b2, b3 = p["b1"], p["b2"], p["b3"]
    aW1, aW2, aW3 = np.abs(W1), np.abs(W2), np.abs(W3)
    slack = 1e-14  # the oracle's own FP64 rounding, relative to the terms
    T1 = np.abs(Xb) @ aW1.T + np.abs(b1)
    e1 = (gamma(9) + slack) * T1
    eH1 = _rounded(Z1, e1, relu=True)
    T2 = (np.abs(H1) + eH1) @ aW2.T + np.abs(b2)
    e2 = eH1 @ aW2.T + (gamma(65) + slack) * T2
    eH2 = _rounded(Z2, e2, relu=True)
    T3 = ((np.abs(H2) + eH2) @ aW3.T)[:, 0] + np.abs(b3[0])
    eout = (eH2 @ aW3.T)[:, 0] + (gamma(65) + slack) * T3
    state = dict(cache=cache, e1=e1, eH1=eH1, e2=e2, eH2=eH2, eout=eout, out=out)
    return out, eout, state


def backward_bound(state, d, ed):
    """(gradient flat [4801], radius flat) for upstream d [N] with radius ed."""
    Xb, Z1, H1, Z2, H2, W1, W2, W3 = state["cache"]
    e1, eH1, e2, eH2 = state["e1"], state["eH1"], state["e2"], state["eH2"]
    parts = {}
    grad = S.mlp_backward(state["cache"], d, parts=parts)
    n = d.shape[0]
    gN = gamma(n) + 1e-14
    aW2, aW3 = np.abs(W2), np.abs(W3[0])
    d3b = parts["d3b"]
    ed3b = _rounded(np.asarray(d, np.float64), ed, relu=False)
    A3 = np.abs(d3b) + ed3b
    aH2, aH1 = np.abs(H2) + eH2, np.abs(H1) + eH1
    e_W3 = np.abs(d3b) @ eH2 + ed3b @ aH2 + gN * (A3 @ aH2)
    e_b3 = np.array([ed.sum() + gN * (np.abs(d) + ed).sum()])
    v2 = d3b[:, None] * W3[0][None, :]
    ev2 = ed3b[:, None] * aW3[None, :]
    edZ2 = _mask_err(Z2, e2, v2, ev2)
    dZ2 = parts["dZ2"]
    edZ2b = _rounded(dZ2, edZ2, relu=False)
    dZ2b = parts["dZ2b"]
    e_b2 = edZ2.sum(0) + gN * (np.abs(dZ2) + edZ2).sum(0)
    aZ2b = np.abs(dZ2b) + edZ2b
    e_W2 = np.abs(dZ2b).T @ eH1 + edZ2b.T @ aH1 + gN * (aZ2b.T @ aH1)
    dH1 = parts["dH1"]
    edH1 = edZ2b @ aW2 + (gamma(64) + 1e-14) * (aZ2b @ aW2)
    edZ1 = _mask_err(Z1, e1, dH1, edH1)
    dZ1 = parts["dZ1"]
    edZ1b = _rounded(dZ1, edZ1, relu=False)
    dZ1b = parts["dZ1b"]
    e_b1 = edZ1.sum(0) + gN * (np.abs(dZ1) + edZ1).sum(0)
    aXb = np.abs(Xb)
    e_W1 = edZ1b.T @ aXb + gN * ((np.abs(dZ1b) + edZ1b).T @ aXb)
    err = S.pack({"W1": e_W1, "b1": e_b1, "W2": e_W2, "b2": e_b2, "W3": e_W3[None, :],
                  "b3": e_b3})
    return grad, err


def pinball_upstream(state, labels, q):
    """The pinball loss's d loss / d prediction per row (the oracle's) with
    its radius on the GPU: rows whose label lies within the prediction's
    radius may take either branch; FP32 forms q and 1/n with rounding."""
    out, eout = state["out"], state["eout"]
    labels = np.asarray(labels, np.float64)
    n = labels.size
    _, d = S.pinball(out, labels, q)
    unc = np.abs(labels - out) <= eout
    ed = np.abs(d) * 4 * U + np.where(unc, 1.0 / n, 0.0)
    return d, ed
