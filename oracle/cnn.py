"""CPU reference of the learned warm start (TEST INFRASTRUCTURE ONLY: used by tests/ and nothing else).

The network is not part of the paper; it predicts an initial iterate for the spatial solves of the
implicit Euler steps (Sec. 2, eq:los) from the current coefficients and the source.  Definition:

* grid: the (n+p) x (n+p) tensor-product coefficient grid (the Dirichlet ring of coefficients is zero);
* input planes (pack): u_k / s_u; e / s_e with e = (w F - kappa dt K u_k) / m, the residual b - A u_k of the
  step's equation at the previous point divided by the row-sum-lumped mass m (the explicit increment in
  coefficient space; w is the step's source weight); and the constant ln(kappa dt n^2) / 4; s_u = rms(u_k),
  s_e = rms(e) over the interior (1 when zero);
* four 3x3 cross-correlations with zero padding, channels 3 -> 32 -> 32 -> 32 -> 1, bias, ReLU after the
  first three; the output y is the increment in units of s_e: guess = u_k + s_e y on the interior;
* training target t = (u_{k+1} - u_k) / s_e, loss = mean over samples and interior points of (y - t)^2.
  The increment of an implicit step is A^{-1} applied to that residual, a smoothed version of e, so the
  target is of order one whatever the state's size.

Parameters are one flat float array, layer by layer: weights [cout][cin][3][3] then bias [cout].

`round_bf16=True` reproduces the rounding points of the GPU kernels (BF16 storage, wide accumulation):
weights, input planes, the three hidden activations and the three back-propagated hidden gradients are
rounded to bfloat16 (round to nearest even); everything else stays in float64 here.  With
`round_bf16=False` everything is float64 and the gradients are the exact gradients of the loss.
"""
from __future__ import annotations

import numpy as np

CH = [3, 32, 32, 32, 1]


def nparams() -> int:
    return sum(CH[l + 1] * CH[l] * 9 + CH[l + 1] for l in range(4))


def unflatten(theta):
    out, o = [], 0
    for l in range(4):
        ci, co = CH[l], CH[l + 1]
        W = np.asarray(theta[o:o + co * ci * 9], dtype=np.float64).reshape(co, ci, 3, 3)
        o += co * ci * 9
        b = np.asarray(theta[o:o + co], dtype=np.float64)
        o += co
        out.append((W, b))
    return out


def flatten(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16(x):
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def conv3x3(a, W, b=None):
    """z[n, co, y, x] = b[co] + sum_ci sum_{dy,dx} W[co, ci, dy+1, dx+1] a[n, ci, y+dy, x+dx], zero outside."""
    nb, ci, G, _ = a.shape
    ap = np.zeros((nb, ci, G + 2, G + 2))
    ap[:, :, 1:-1, 1:-1] = a
    z = np.zeros((nb, W.shape[0], G, G))
    for dy in range(3):
        for dx in range(3):
            win = ap[:, :, dy:dy + G, dx:dx + G]
            z += np.einsum("oc,ncyx->noyx", W[:, :, dy, dx], win)
    if b is not None:
        z += b[None, :, None, None]
    return z


def conv3x3_transpose(g, W):
    """Adjoint of conv3x3 in its input: d[n, ci, y, x] = sum_co sum_{dy,dx} W[co, ci, dy+1, dx+1] g[n, co, y-dy, x-dx]."""
    nb, co, G, _ = g.shape
    gp = np.zeros((nb, co, G + 2, G + 2))
    gp[:, :, 1:-1, 1:-1] = g
    d = np.zeros((nb, W.shape[1], G, G))
    for dy in range(3):
        for dx in range(3):
            # g[y - (dy-1)] = gp[y - dy + 2]
            win = gp[:, :, 2 - dy:2 - dy + G, 2 - dx:2 - dx + G]
            d += np.einsum("oc,noyx->ncyx", W[:, :, dy, dx], win)
    return d


def conv3x3_wgrad(a, g):
    """dW[co, ci, dy+1, dx+1] = sum_n sum_{y,x} g[n, co, y, x] a[n, ci, y+dy, x+dx] (zero outside)."""
    nb, ci, G, _ = a.shape
    ap = np.zeros((nb, ci, G + 2, G + 2))
    ap[:, :, 1:-1, 1:-1] = a
    dW = np.zeros((g.shape[1], ci, 3, 3))
    for dy in range(3):
        for dx in range(3):
            dW[:, :, dy, dx] = np.einsum("noyx,ncyx->oc", g, ap[:, :, dy:dy + G, dx:dx + G])
    return dW


def forward(theta, x, round_bf16=False):
    """x: (nb, 3, G, G).  Returns y (nb, G, G) and the activations needed by backward."""
    r = bf16 if round_bf16 else (lambda v: np.asarray(v, dtype=np.float64))
    layers = [(r(W), np.asarray(b, np.float64)) for W, b in unflatten(theta)]
    acts = [r(x)]
    for l in range(3):
        W, b = layers[l]
        acts.append(r(np.maximum(conv3x3(acts[-1], W, b), 0.0)))
    W, b = layers[3]
    y = conv3x3(acts[-1], W, b)[:, 0]
    return y, (layers, acts)


def interior_mask(G):
    m = np.zeros((G, G))
    m[1:-1, 1:-1] = 1.0
    return m


def loss_and_grad(theta, x, t, round_bf16=False):
    """Mean squared error over samples and interior points, and its gradient in the flat layout."""
    y, (layers, acts) = forward(theta, x, round_bf16)
    r = bf16 if round_bf16 else (lambda v: v)
    nb, G, _ = y.shape
    m = interior_mask(G)[None]
    cnt = nb * (G - 2) ** 2
    e = (y - t) * m
    loss = float(np.sum(e * e) / cnt)
    g = (2.0 / cnt * e)[:, None]  # dL/dy, zero on the Dirichlet ring
    grads = [None] * 4
    for l in (3, 2, 1, 0):
        W, _ = layers[l]
        grads[l] = (conv3x3_wgrad(acts[l], g), g.sum(axis=(0, 2, 3)))
        if l > 0:
            g = r(conv3x3_transpose(g, W) * (acts[l] > 0))
    return loss, flatten(grads)


def pack(u, F, mlp, K, w, kdt, n, p, u_next=None):
    """Input planes of one sample and (optionally) its training target.

    u, F, mlp, u_next: interior vectors of length (n+p-2)^2, x fastest; K: the interior stiffness matrix
    (dense or scipy sparse); w: the step's source weight; kdt: kappa dt.  Returns (x (3, G, G), s_e,
    t (G, G))."""
    G = n + p
    nin = G - 2
    u = np.asarray(u, np.float64)
    e = (w * np.asarray(F, np.float64) - kdt * (K @ u)) / np.asarray(mlp, np.float64)
    s_u = np.sqrt(np.mean(u * u))
    s_e = np.sqrt(np.mean(e * e))
    s_u = s_u if s_u != 0.0 else 1.0
    s_e = s_e if s_e != 0.0 else 1.0
    x = np.zeros((3, G, G))
    x[0, 1:-1, 1:-1] = (u / s_u).reshape(nin, nin)
    x[1, 1:-1, 1:-1] = (e / s_e).reshape(nin, nin)
    x[2, :, :] = np.log(kdt * n * n) / 4.0
    t = None
    if u_next is not None:
        t = np.zeros((G, G))
        t[1:-1, 1:-1] = ((np.asarray(u_next, np.float64) - u) / s_e).reshape(nin, nin)
    return x, s_e, t


def unpack(y, u, s):
    """guess = u + s y on the interior."""
    return np.asarray(u, np.float64) + s * np.asarray(y, np.float64)[1:-1, 1:-1].ravel()


def adam(theta, grad, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba), bias-corrected, returning new (theta, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
