"""FP64 CPU oracle of the warm-start network's layers — TEST INFRASTRUCTURE.

Plain definitions, NHWC activations (n, y, x, c), direct sums:

  conv3x3      y[n,i,j,o] = b[o] + sum_{dy,dx,c} W[o,dy,dx,c] x[n, i+dy-1, j+dx-1, c]
               (zero padding), optional ReLU
  conv3x3 grads  dx = transposed correlation, dW[o,dy,dx,c] = sum_{n,i,j} dy[n,i,j,o]
               x[n,i+dy-1,j+dx-1,c], db[o] = sum dy[..., o]
  maxpool2     y[n,i,j,c] = max over the 2x2 block; gradient to the first maximum in
               (0,0), (0,1), (1,0), (1,1) order
  up2          nearest-neighbour 2x upsampling; gradient = sum over the 2x2 block
  conv1x1      y[n,i,j] = b + sum_c w[c] x[n,i,j,c]
  mse          mean((y - t)^2) and its gradient 2 (y - t) / numel
  adam         Kingma & Ba (2015) update with bias correction
  bf16         round-to-nearest-even to bfloat16 (to feed the exact values a bf16 matrix
               core consumes)

The network composition follows the 4-level U-Net (Ronneberger et al. 2015) with
nearest upsampling and channel concatenation; `unet_forward` / `unet_loss_grad` run it in
FP64 for the end-to-end gradient check.
"""
from __future__ import annotations

import numpy as np


def bf16(a: np.ndarray) -> np.ndarray:
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.ascontiguousarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def conv3x3(x, w, b=None, relu=False):
    """x [N,H,W,C], w [O,3,3,C] -> [N,H,W,O]."""
    x = np.asarray(x, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((n, h, wd, w.shape[0]))
    for dy in range(3):
        for dx in range(3):
            y += xp[:, dy:dy + h, dx:dx + wd, :] @ w[:, dy, dx, :].T
    if b is not None:
        y += np.asarray(b, dtype=np.float64)
    return np.maximum(y, 0.0) if relu else y


def conv3x3_grad_input(dy, w, shape):
    """Gradient of sum(dy * conv3x3(x, w)) with respect to x."""
    dy = np.asarray(dy, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    n, h, wd, c = shape
    dxp = np.zeros((n, h + 2, wd + 2, c))
    for a in range(3):
        for b in range(3):
            dxp[:, a:a + h, b:b + wd, :] += dy @ w[:, a, b, :]
    return dxp[:, 1:-1, 1:-1]


def conv3x3_grad_weight(x, dy):
    """dW[o,dy,dx,c] = sum_{n,i,j} dy[n,i,j,o] x[n,i+dy-1,j+dx-1,c]; db[o] = sum dy."""
    x = np.asarray(x, dtype=np.float64)
    dy = np.asarray(dy, dtype=np.float64)
    n, h, wd, c = x.shape
    xp = np.zeros((n, h + 2, wd + 2, c))
    xp[:, 1:-1, 1:-1] = x
    o = dy.shape[-1]
    dw = np.zeros((o, 3, 3, c))
    d2 = dy.reshape(-1, o)
    for a in range(3):
        for b in range(3):
            dw[:, a, b, :] = d2.T @ xp[:, a:a + h, b:b + wd, :].reshape(-1, c)
    return dw, d2.sum(axis=0)


def maxpool2(x):
    x = np.asarray(x, dtype=np.float64)
    n, h, w, c = x.shape
    return x.reshape(n, h // 2, 2, w // 2, 2, c).max(axis=(2, 4))


def maxpool2_grad(x, dy):
    x = np.asarray(x, dtype=np.float64)
    n, h, w, c = x.shape
    dx = np.zeros_like(x)
    m = maxpool2(x)
    taken = np.zeros(m.shape, dtype=bool)
    for a in range(2):
        for b in range(2):
            hit = (x[:, a::2, b::2, :] == m) & ~taken
            dx[:, a::2, b::2, :] = np.where(hit, dy, 0.0)
            taken |= hit
    return dx


def up2(x):
    x = np.asarray(x, dtype=np.float64)
    return x.repeat(2, axis=1).repeat(2, axis=2)


def up2_grad(dy):
    dy = np.asarray(dy, dtype=np.float64)
    n, h, w, c = dy.shape
    return dy.reshape(n, h // 2, 2, w // 2, 2, c).sum(axis=(2, 4))


def conv1x1(x, w, b):
    return np.asarray(x, dtype=np.float64) @ np.asarray(w, dtype=np.float64) + float(b)


def mse(y, t):
    y = np.asarray(y, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    d = y - t
    return float(np.mean(d * d)), 2.0 * d / d.size


def adam(p, g, m, v, step, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (step counts from 1); returns (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return p - lr * mh / (np.sqrt(vh) + eps), m, v


# ----------------------------------------------------------------------------- network

def unet_channels(levels=4, base=32):
    return [base * (2 ** l) for l in range(levels)]


def unet_param_shapes(levels=4, base=32, in_ch=4):
    """(name, shape) of every parameter in a fixed order: per 3x3 conv its weight [O,3,3,C]
    then bias [O]; the 1x1 head weight [C] and bias []."""
    ch = unet_channels(levels, base)
    shapes = []
    prev = in_ch
    for l in range(levels):
        shapes += [(f"enc{l}a.w", (ch[l], 3, 3, prev)), (f"enc{l}a.b", (ch[l],)),
                   (f"enc{l}b.w", (ch[l], 3, 3, ch[l])), (f"enc{l}b.b", (ch[l],))]
        prev = ch[l]
    for l in range(levels - 2, -1, -1):
        cin = ch[l + 1] + ch[l]
        shapes += [(f"dec{l}a.w", (ch[l], 3, 3, cin)), (f"dec{l}a.b", (ch[l],)),
                   (f"dec{l}b.w", (ch[l], 3, 3, ch[l])), (f"dec{l}b.b", (ch[l],))]
    shapes += [("head.w", (ch[0],)), ("head.b", ())]
    return shapes


def unpack(flat, levels=4, base=32, in_ch=4):
    out, o = {}, 0
    for name, shp in unet_param_shapes(levels, base, in_ch):
        k = int(np.prod(shp)) if shp else 1
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def unet_forward(x, P, levels=4, round_bf16=False):
    """x [N,H,W,in_ch]; P from unpack.  With round_bf16 every 3x3-conv operand (weights and
    input activation) is rounded to bfloat16 first, as the matrix-core kernels consume it.
    Returns (output [N,H,W], tape)."""
    q = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    tape = {"x": x}
    h = x
    skips = []
    for l in range(levels):
        if l > 0:
            h = maxpool2(h)
            tape[f"pool{l}"] = h
        tape[f"enc{l}a.in"] = h
        h = conv3x3(q(h), q(P[f"enc{l}a.w"]), P[f"enc{l}a.b"], relu=True)
        tape[f"enc{l}b.in"] = h
        h = conv3x3(q(h), q(P[f"enc{l}b.w"]), P[f"enc{l}b.b"], relu=True)
        tape[f"enc{l}.out"] = h
        skips.append(h)
    for l in range(levels - 2, -1, -1):
        u = up2(h)
        c = np.concatenate([u, skips[l]], axis=-1)
        tape[f"dec{l}a.in"] = c
        h = conv3x3(q(c), q(P[f"dec{l}a.w"]), P[f"dec{l}a.b"], relu=True)
        tape[f"dec{l}b.in"] = h
        h = conv3x3(q(h), q(P[f"dec{l}b.w"]), P[f"dec{l}b.b"], relu=True)
        tape[f"dec{l}.out"] = h
    tape["head.in"] = h
    y = conv1x1(h, P["head.w"], P["head.b"])
    return y, tape


def unet_loss(x, t, flat, levels=4, base=32, in_ch=4):
    P = unpack(flat, levels, base, in_ch)
    y, _ = unet_forward(x, P, levels)
    return mse(y, t)[0]


def unet_loss_grad(x, t, flat, levels=4, base=32, in_ch=4, round_bf16=False):
    """FP64 reverse pass through the network, composed from the layer gradients above.
    With round_bf16 the operands of every 3x3-convolution product are rounded to bfloat16
    where a bf16 matrix core consumes them: forward (input activation, weights), input
    gradient (output gradient, weights), weight gradient (input activation, output
    gradient).  Returns (loss, flat gradient in parameter order)."""
    q = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    P = unpack(flat, levels, base, in_ch)
    y, T = unet_forward(x, P, levels, round_bf16=round_bf16)
    loss, dyv = mse(y, t)
    G = {}
    h = T["head.in"]
    G["head.w"] = np.einsum("nijc,nij->c", h, dyv)
    G["head.b"] = np.array(dyv.sum())
    dh = dyv[..., None] * P["head.w"] * (h > 0)
    ch = unet_channels(levels, base)
    dskip = [None] * levels

    def conv_back(name, dout, need_input=True):
        xin = T[f"{name}.in"]
        dw, db = conv3x3_grad_weight(q(xin), q(dout))
        G[f"{name}.w"], G[f"{name}.b"] = dw, db
        if not need_input:
            return None
        return conv3x3_grad_input(q(dout), q(P[f"{name}.w"]), xin.shape) * (xin > 0)

    for l in range(levels - 1):
        dh = conv_back(f"dec{l}b", dh)
        dc = conv_back(f"dec{l}a", dh)
        dskip[l] = dc[..., ch[l + 1]:]
        dh = up2_grad(dc[..., :ch[l + 1]])
    for l in range(levels - 1, -1, -1):
        dh = conv_back(f"enc{l}b", dh)
        if l == 0:
            conv_back(f"enc{l}a", dh, need_input=False)
            break
        dp = conv_back(f"enc{l}a", dh)
        dh = maxpool2_grad(T[f"enc{l - 1}.out"], dp) + dskip[l - 1]
    grads = [np.asarray(G[name]).reshape(-1) for name, _ in unet_param_shapes(levels, base, in_ch)]
    return loss, np.concatenate(grads)
