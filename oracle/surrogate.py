"""FP64 reference of the learned overlap surrogate.

TEST INFRASTRUCTURE ONLY (same rule as the rest of this package).

The surrogate is an addition to the paper.  For a tetrahedron whose bounding
box spans at most 2 cells per axis it predicts the overlap fractions
|T cap C| / |T| of the cell average of Eq. (1) for the 2x2x2 cells starting at
the bbox origin lo = floor(min v):

    x  (12)  = the 4 vertices minus lo, in cell units, split-vertex order
    h1 = silu(W1 x  + b1)     W1: 64 x 12
    h2 = silu(W2 h1 + b2)     W2: 64 x 64
    h3 = silu(W3 h2 + b3)     W3: 64 x 64
    z  =      W4 h3 + b4      W4:  8 x 64
    p  = softmax of z over the cells inside [lo, hi] (mask); 0 elsewhere

Cell c = 4 dx + 2 dy + dz.  The network sees the tetrahedron in a canonical
pose (canonical()): the fractions do not change when the vertices are
listed in another order, and reflecting a straddling axis (x -> 2 - x for an
axis whose bbox spans 2 cells) only swaps that axis's cells.  So every
straddling axis whose vertex sum exceeds 4 (centroid beyond the middle
plane) is reflected, the vertices are sorted lexicographically, and the
network's output for canonical cell c' is the prediction for cell c' ^ r,
r = the reflected axes' cell bits.  Parameters are one packed vector (LAYOUT below,
matrices row-major [out][in]).  The matrices are used rounded to bfloat16;
the biases stay float32.  This reference evaluates the network in float64 on
those rounded values; training minimises the soft-label cross entropy
-sum_c y_c log p_c averaged over the batch, with Adam (Kingma & Ba 2015).
"""

from __future__ import annotations

import numpy as np

HIDDEN = 64
N_IN = 12
N_OUT = 8

# (name, shape) in storage order
LAYOUT = [
    ("W1", (HIDDEN, N_IN)), ("b1", (HIDDEN,)),
    ("W2", (HIDDEN, HIDDEN)), ("b2", (HIDDEN,)),
    ("W3", (HIDDEN, HIDDEN)), ("b3", (HIDDEN,)),
    ("W4", (N_OUT, HIDDEN)), ("b4", (N_OUT,)),
]
N_PARAMS = sum(int(np.prod(s)) for _, s in LAYOUT)  # 9672


def unpack(theta: np.ndarray) -> dict:
    out, o = {}, 0
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        out[name] = theta[o:o + n].reshape(shape)
        o += n
    return out


def pack(params: dict) -> np.ndarray:
    return np.concatenate([np.asarray(params[name], dtype=np.float64).reshape(-1)
                           for name, _ in LAYOUT])


def bf16_round(a) -> np.ndarray:
    """float32 -> nearest bfloat16 value (ties to even), returned as float32.

    bfloat16 keeps the top 16 bits of the float32 encoding; rounding adds
    0x7FFF plus the lowest kept bit before truncating (finite inputs)."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def effective(theta_fp32: np.ndarray) -> np.ndarray:
    """The values the network computes with: matrices rounded to bfloat16, biases float32."""
    theta = np.asarray(theta_fp32, dtype=np.float32)
    out = theta.astype(np.float64).copy()
    o = 0
    for name, shape in LAYOUT:
        n = int(np.prod(shape))
        if name.startswith("W"):
            out[o:o + n] = bf16_round(theta[o:o + n]).astype(np.float64)
        o += n
    return out


def mask_bits(mask: np.ndarray) -> np.ndarray:
    """uint8 cell masks -> bool [n, 8] (bit c = cell c)."""
    m = np.asarray(mask, dtype=np.uint8)[:, None]
    return ((m >> np.arange(N_OUT, dtype=np.uint8)[None, :]) & 1).astype(bool)


AXIS_BIT = (4, 2, 1)  # cell-index bit of each axis


def canonical(x: np.ndarray, mask: np.ndarray):
    """Canonical pose: (features float32 [n, 12], r int [n]).

    An axis a is reflected iff its bbox spans 2 cells (mask bit AXIS_BIT[a] set)
    and ((x0 + x1) + x2) + x3 > 4 in float64 over the 4 vertices' coordinate a;
    reflected coordinates are 2 - x in float32; the 4 vertices are then sorted
    lexicographically by (x, y, z)."""
    v = np.array(x, dtype=np.float32).reshape(-1, 4, 3)
    m = np.asarray(mask, dtype=np.int64)
    r = np.zeros(len(v), dtype=np.int64)
    for a in range(3):
        s = ((v[:, 0, a].astype(np.float64) + v[:, 1, a]) + v[:, 2, a]) + v[:, 3, a]
        refl = (((m >> AXIS_BIT[a]) & 1) == 1) & (s > 4.0)
        v[:, :, a] = np.where(refl[:, None], np.float32(2.0) - v[:, :, a], v[:, :, a])
        r |= np.where(refl, AXIS_BIT[a], 0)
    order = np.lexsort((v[:, :, 2], v[:, :, 1], v[:, :, 0]), axis=1)
    v = np.take_along_axis(v, order[:, :, None], 1)
    return v.reshape(-1, 12), r


def to_canonical_cells(a: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Per-cell values a[n, 8] in the original order -> canonical order (c' holds c' ^ r)."""
    idx = np.arange(N_OUT)[None, :] ^ np.asarray(r)[:, None]
    return np.take_along_axis(np.asarray(a), idx, 1)


def from_canonical_cells(a: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Inverse of to_canonical_cells (the map is an involution)."""
    return to_canonical_cells(a, r)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_grad(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta: np.ndarray, x: np.ndarray, mask: np.ndarray):
    """Probabilities p [n, 8] (original cell order) and the intermediates of the
    network on the canonical pose (z1..z4, h1..h3, canonical probabilities)."""
    xc, r = canonical(x, mask)
    pc, c = net(theta, xc, mask)
    c["r"] = r
    c["pc"] = pc
    return from_canonical_cells(pc, r), c


def net(theta: np.ndarray, x: np.ndarray, mask: np.ndarray):
    """The network on given (canonical) features: probabilities and intermediates.
    The cell mask is the same in both poses."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    z1 = x @ P["W1"].T + P["b1"]
    h1 = silu(z1)
    z2 = h1 @ P["W2"].T + P["b2"]
    h2 = silu(z2)
    z3 = h2 @ P["W3"].T + P["b3"]
    h3 = silu(z3)
    z4 = h3 @ P["W4"].T + P["b4"]
    mb = mask_bits(mask)
    zm = np.where(mb, z4, -np.inf)
    zmax = zm.max(axis=1, keepdims=True)
    e = np.where(mb, np.exp(zm - zmax), 0.0)
    p = e / e.sum(axis=1, keepdims=True)
    return p, {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2, "z3": z3, "h3": h3, "z4": z4,
               "mb": mb, "P": P}


def loss(theta, x, y, mask) -> float:
    """Mean over the batch of -sum_c y_c log p_c (masked-out cells carry y = 0)."""
    p, c = forward(theta, x, mask)
    y = np.asarray(y, dtype=np.float64)
    lp = np.where(c["mb"], np.log(np.where(c["mb"], p, 1.0)), 0.0)
    return float(-(y * lp).sum() / x.shape[0])


def backward(theta, x, y, mask):
    """(loss, gradient of the mean loss with respect to theta) by reverse mode.
    The loss is the same in the canonical pose with the labels permuted alike."""
    xc, r = canonical(x, mask)
    return net_backward(theta, xc, to_canonical_cells(np.asarray(y, dtype=np.float64), r), mask)


def net_backward(theta, x, y, mask):
    """(loss, gradient) of the network on given (canonical) features and labels."""
    p, c = net(theta, x, mask)
    P = c["P"]
    n = x.shape[0]
    y = np.asarray(y, dtype=np.float64)
    lp = np.where(c["mb"], np.log(np.where(c["mb"], p, 1.0)), 0.0)
    L = float(-(y * lp).sum() / n)
    # d/dz of -sum y log softmax(z) over the masked-in cells is p * sum(y) - y
    dz4 = np.where(c["mb"], p * y.sum(axis=1, keepdims=True) - y, 0.0) / n
    g = {"W4": dz4.T @ c["h3"], "b4": dz4.sum(0)}
    dz3 = (dz4 @ P["W4"]) * silu_grad(c["z3"])
    g["W3"], g["b3"] = dz3.T @ c["h2"], dz3.sum(0)
    dz2 = (dz3 @ P["W3"]) * silu_grad(c["z2"])
    g["W2"], g["b2"] = dz2.T @ c["h1"], dz2.sum(0)
    dz1 = (dz2 @ P["W2"]) * silu_grad(c["z1"])
    g["W1"], g["b1"] = dz1.T @ c["x"], dz1.sum(0)
    return L, pack(g)


def adam(theta, grad, m, v, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
         eps: float = 1e-8):
    """One Adam update (bias-corrected moments); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def bbox_overlap_fractions(x: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """Non-learned baseline: each cell's share of the tetrahedron's bounding box."""
    v = np.asarray(x, dtype=np.float64).reshape(-1, 4, 3)
    lo, hi = v.min(axis=1), v.max(axis=1)
    out = np.ones((v.shape[0], N_OUT))
    for c in range(N_OUT):
        d = np.array([(c >> 2) & 1, (c >> 1) & 1, c & 1], dtype=np.float64)
        ov = np.clip(np.minimum(hi, d + 1.0) - np.maximum(lo, d), 0.0, None)
        ext = np.maximum(hi - lo, 0.0)
        # a flat axis puts all of that axis in the cell that holds it
        flat = ext == 0.0
        ov = np.where(flat, ((lo >= d) & (lo < d + 1.0)).astype(np.float64), ov)
        ext = np.where(flat, 1.0, ext)
        out[:, c] = np.prod(ov / ext, axis=1)
    return np.where(mask_bits(mask), out, 0.0)
