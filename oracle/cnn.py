"""Plain numpy (float64) oracle of the learned initial-plane proposal.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU-baseline leg
of the benchmark, never by the library or its binding.

The paper proposes no network; it states only that the search starts from random planes
(Sec. III-B: random depth within the depth range, random normal) and that a good start
speeds up convergence.  The network here is the library's own addition, so this oracle
is written from the definition of each operation, with no blocking, fusion or
reordering:

* 3x3 convolution with zero padding, tap t = 3 (dy + 1) + (dx + 1) reading the input
  at (y + dy, x + dx), weights w[t][cin][cout] plus a bias per output channel;
* 5 layers 5 -> 32 -> 32 -> 32 -> 32 -> 4, ReLU after the first four;
* loss per pixel (mask m): m (|log d - log d_t| + lambda (1 - n . n_t)) with
  d = lo + (hi - lo) sigmoid(o0) and n = o[1:4] / |o[1:4]| (+1e-6 in the norm), summed and
  divided by the number of pixels;
* the gradient by the chain rule, layer by layer (a textbook backward pass);
* Adam (Kingma & Ba, 2015) with bias correction.

The GPU stores weights, activations and back-propagated gradients as bfloat16.  The
``like_gpu`` options round exactly the quantities the GPU stores (round to nearest even,
the format's definition) so the two can be compared closely; with the options off
everything is float64.  The proposal input builder, the decoding of the outputs into
planes and the training targets are here too (see their docstrings).
"""
from __future__ import annotations

import numpy as np

SHAPES = ((5, 32), (32, 32), (32, 32), (32, 32), (32, 4))


def param_count() -> int:
    return sum(9 * ci * co + co for ci, co in SHAPES)


def unpack(flat):
    """flat parameter vector -> [(w (9, cin, cout), b (cout,))] per layer."""
    flat = np.asarray(flat, dtype=np.float64)
    out, o = [], 0
    for ci, co in SHAPES:
        w = flat[o:o + 9 * ci * co].reshape(9, ci, co)
        o += 9 * ci * co
        b = flat[o:o + co]
        o += co
        out.append((w, b))
    assert o == flat.size
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([w.ravel(), b.ravel()]) for w, b in layers])


def bf16(x):
    """Round float32 values to bfloat16 (nearest, ties to even) and return them as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return (u.astype(np.uint32)).view(np.float32).astype(np.float64)


def f32(x):
    return np.asarray(x, dtype=np.float32).astype(np.float64)


def conv3x3(x, w, b=None):
    """x (B, h, w, cin), w (9, cin, cout) -> (B, h, w, cout); zero outside the image."""
    B, h, wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.zeros((B, h, wd, w.shape[2]))
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        y += np.tensordot(xp[:, 1 + dy:1 + dy + h, 1 + dx:1 + dx + wd, :], w[t], axes=([3], [0]))
    if b is not None:
        y += b
    return y


def conv3x3_wgrad(x, g):
    """dL/dw[t] = sum over pixels of x(p + off_t) g(p)^T -> (9, cin, cout)."""
    B, h, wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = []
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        xs = xp[:, 1 + dy:1 + dy + h, 1 + dx:1 + dx + wd, :]
        out.append(np.tensordot(xs, g, axes=([0, 1, 2], [0, 1, 2])))
    return np.stack(out)


def conv3x3_dgrad(g, w):
    """dL/dx(q) = sum_t w[t] g(q - off_t) -> (B, h, w, cin)."""
    B, h, wd, _ = g.shape
    gp = np.pad(g, ((0, 0), (1, 1), (1, 1), (0, 0)))
    out = np.zeros((B, h, wd, w.shape[1]))
    for t in range(9):
        dy, dx = t // 3 - 1, t % 3 - 1
        out += np.tensordot(gp[:, 1 - dy:1 - dy + h, 1 - dx:1 - dx + wd, :], w[t], axes=([3], [1]))
    return out


def forward(params, x, like_gpu: bool = False):
    """-> (output (B, h, w, 4), activations [input, a1, .., a4]) for x (B, h, w, 5)."""
    layers = unpack(params)
    a = bf16(x) if like_gpu else np.asarray(x, dtype=np.float64)
    acts = [a]
    for i, (w, b) in enumerate(layers):
        if like_gpu:
            w, b = bf16(w), f32(b)
        z = conv3x3(a, w, b)
        if i < len(layers) - 1:
            a = np.maximum(z, 0.0)
            if like_gpu:
                a = bf16(a)
            acts.append(a)
        else:
            out = f32(z) if like_gpu else z
    return out, acts


def decode_depth_normal(out, drange):
    """Raw outputs (B, h, w, 4), depth ranges (B, 2) -> depth (B, h, w), unit normal (B, h, w, 3)."""
    lo = drange[:, 0][:, None, None]
    hi = drange[:, 1][:, None, None]
    s = 1.0 / (1.0 + np.exp(-out[..., 0]))
    d = lo + (hi - lo) * s
    v = out[..., 1:4]
    nrm = np.sqrt((v * v).sum(-1)) + 1e-6
    return d, v / nrm[..., None]


def loss(out, target, mask, drange, lam: float = 1.0) -> float:
    d, n = decode_depth_normal(out, np.asarray(drange, dtype=np.float64))
    per = np.abs(np.log(d) - np.log(target[..., 0])) + lam * (1.0 - (n * target[..., 1:4]).sum(-1))
    return float((mask * per).sum() / mask.size)


def loss_output_grad(out, target, mask, drange, lam: float = 1.0):
    """dL/d(output) by the chain rule: the sign of the log-depth error through the sigmoid,
    and the projection of -lambda n_t onto the tangent space of the normalisation."""
    drange = np.asarray(drange, dtype=np.float64)
    lo = drange[:, 0][:, None, None]
    hi = drange[:, 1][:, None, None]
    s = 1.0 / (1.0 + np.exp(-out[..., 0]))
    d = lo + (hi - lo) * s
    diff = np.log(d) - np.log(target[..., 0])
    m = mask / mask.size
    g = np.zeros_like(out)
    g[..., 0] = m * np.sign(diff) * (hi - lo) * s * (1.0 - s) / d
    v = out[..., 1:4]
    nrm = np.sqrt((v * v).sum(-1)) + 1e-6
    n = v / nrm[..., None]
    dot = (n * target[..., 1:4]).sum(-1)
    g[..., 1:4] = (-m * lam / nrm)[..., None] * (target[..., 1:4] - dot[..., None] * n)
    return g


def loss_grad(params, x, target, mask, drange, lam: float = 1.0, like_gpu: bool = False):
    """-> (loss, flat gradient).  like_gpu also rounds the back-propagated gradients to
    bfloat16 where the GPU stores them (the output gradient and each layer's input gradient)."""
    layers = unpack(params)
    out, acts = forward(params, x, like_gpu)
    L = loss(out, target, mask, drange, lam)
    g = loss_output_grad(out, target, mask, drange, lam)
    if like_gpu:
        g = bf16(g)
    grads = [None] * len(layers)
    for i in range(len(layers) - 1, -1, -1):
        w, _ = layers[i]
        grads[i] = (conv3x3_wgrad(acts[i], g), g.sum(axis=(0, 1, 2)))
        if i == 0:
            break
        gx = conv3x3_dgrad(g, bf16(w) if like_gpu else w)
        gx = gx * (acts[i] > 0)
        g = bf16(gx) if like_gpu else gx
    return L, pack(grads)


def adam(params, grad, m, v, t: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam step -> (params, m, v)."""
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------------------- proposal

def camera_centre(R, t):
    return -np.asarray(R, dtype=np.float64).T @ np.asarray(t, dtype=np.float64)


def nearest_sources(R, t, ref, srcs, k: int = 4):
    """The k sources of srcs whose camera centres are closest to the reference's (ties: list order)."""
    c0 = camera_centre(R[ref], t[ref])
    d2 = [float(((camera_centre(R[s], t[s]) - c0) ** 2).sum()) for s in srcs]
    order = sorted(range(len(srcs)), key=lambda i: (d2[i], i))
    return [srcs[i] for i in order[:k]]


def plane_homography(K0, R0, t0, K1, R1, t1, depth):
    """Reference pixel -> source pixel for the points at reference depth Z = depth."""
    Rr = R1 @ R0.T
    tr = t1 - Rr @ t0
    A = Rr + np.outer(tr, np.array([0.0, 0.0, 1.0])) / depth
    return K1 @ A @ np.linalg.inv(K0)


def bilinear(img, u, v):
    """Bilinear value of img (H, W) at (u, v) with 0 <= u <= W - 1, 0 <= v <= H - 1."""
    H, W = img.shape
    x0, y0 = int(np.floor(u)), int(np.floor(v))
    x1, y1 = min(x0 + 1, W - 1), min(y0 + 1, H - 1)
    fx, fy = u - x0, v - y0
    top = img[y0, x0] * (1 - fx) + img[y0, x1] * fx
    bot = img[y1, x0] * (1 - fx) + img[y1, x1] * fx
    return top * (1 - fy) + bot * fy


def proposal_inputs(images, K, R, t, depth_range, ref, srcs):
    """Network input (ceil(H/4), ceil(W/4), 5) of reference ``ref``: the mean of each 4x4
    reference block (edge blocks repeat the last row / column), then the four nearest
    sources sampled at H_k (4X + 1.5, 4Y + 1.5, 1) with H_k the homography of the plane
    Z = (d_lo + d_hi) / 2, 0 where the point falls outside a source or behind it; grey
    values g enter as (g - 127.5) / 64."""
    img0 = np.asarray(images[ref], dtype=np.float64)
    H, W = img0.shape
    h, w = (H + 3) // 4, (W + 3) // 4
    out = np.zeros((h, w, 5))
    ys = np.minimum(np.arange(4 * h), H - 1)
    xs = np.minimum(np.arange(4 * w), W - 1)
    big = img0[np.ix_(ys, xs)]
    out[..., 0] = (big.reshape(h, 4, w, 4).mean(axis=(1, 3)) - 127.5) / 64.0
    dmid = 0.5 * (depth_range[0] + depth_range[1])
    for k, s in enumerate(nearest_sources(R, t, ref, srcs)):
        Hm = plane_homography(K[ref], R[ref], t[ref], K[s], R[s], t[s], dmid)
        img = np.asarray(images[s], dtype=np.float64)
        Hs, Ws = img.shape
        for Y in range(h):
            for X in range(w):
                p = Hm @ np.array([4 * X + 1.5, 4 * Y + 1.5, 1.0])
                if p[2] <= 0:
                    continue
                u, v = p[0] / p[2], p[1] / p[2]
                if 0 <= u <= Ws - 1 and 0 <= v <= Hs - 1:
                    out[Y, X, 1 + k] = (bilinear(img, u, v) - 127.5) / 64.0
    return out


def decode(out, K, depth_range, H, W):
    """Full-resolution planes (H, W, 4) from raw outputs (h, w, 4): bilinear upsampling of
    the outputs at ((x - 1.5) / 4, (y - 1.5) / 4) clamped to the grid, depth
    lo + (hi - lo) sigmoid(o0), normal o[1:4] normalised ((0, 0, -1) if zero) and turned
    to face the camera (n . K^-1 (x, y, 1) < 0)."""
    h, w, _ = out.shape
    X = np.clip((np.arange(W) - 1.5) / 4.0, 0, w - 1)
    Y = np.clip((np.arange(H) - 1.5) / 4.0, 0, h - 1)
    x0 = np.floor(X).astype(int)
    y0 = np.floor(Y).astype(int)
    x1 = np.minimum(x0 + 1, w - 1)
    y1 = np.minimum(y0 + 1, h - 1)
    fx = (X - x0)[None, :, None]
    fy = (Y - y0)[:, None, None]
    o = ((out[y0][:, x0] * (1 - fx) + out[y0][:, x1] * fx) * (1 - fy)
         + (out[y1][:, x0] * (1 - fx) + out[y1][:, x1] * fx) * fy)
    lo, hi = depth_range
    d = lo + (hi - lo) / (1.0 + np.exp(-o[..., 0]))
    v = o[..., 1:4]
    nrm = np.sqrt((v * v).sum(-1))
    n = np.where(nrm[..., None] > 1e-6, v / np.maximum(nrm, 1e-300)[..., None], np.array([0.0, 0.0, -1.0]))
    xx, yy = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    rays = np.stack([xx, yy, np.ones_like(xx)], -1) @ np.linalg.inv(K).T
    flip = (n * rays).sum(-1) > 0
    n[flip] = -n[flip]
    return np.concatenate([n, d[..., None]], -1)


def targets(depth, normal, cost, max_cost):
    """Targets (h, w, 4) and mask (h, w): block (X, Y) takes full-resolution pixels
    (4X + 1 .. 4X + 2, 4Y + 1 .. 4Y + 2) (clamped); mask 1 iff all four have depth > 0 and
    cost < max_cost; target = mean depth and normalised mean normal."""
    H, W = depth.shape
    h, w = (H + 3) // 4, (W + 3) // 4
    tgt = np.zeros((h, w, 4))
    tgt[..., 0] = 1.0
    tgt[..., 3] = -1.0
    mask = np.zeros((h, w))
    for Y in range(h):
        for X in range(w):
            ys = [min(4 * Y + dy, H - 1) for dy in (1, 2)]
            xs = [min(4 * X + dx, W - 1) for dx in (1, 2)]
            pix = [(y, x) for y in ys for x in xs]
            ds = np.array([depth[p] for p in pix], dtype=np.float64)
            cs = np.array([cost[p] for p in pix], dtype=np.float64)
            ns = np.array([normal[p] for p in pix], dtype=np.float64).sum(0)
            nn = np.sqrt((ns * ns).sum())
            if (ds > 0).all() and (cs < max_cost).all() and nn > 1e-6:
                mask[Y, X] = 1.0
                tgt[Y, X, 0] = ds.mean()
                tgt[Y, X, 1:] = ns / nn
    return tgt, mask
