"""CPU reference of the screening model (include/reff_surrogate.h).

TEST INFRASTRUCTURE ONLY.  Nothing in the library's product path may import
or call this module; only the tests use it.  It shares no code with the HIP
path: it builds the input channels from the plain descriptor dict, unpacks
the flat parameter vector from the layout the header documents, and runs
the network with stock PyTorch CPU operators in float64 (autograd supplies
the reference gradients).

The paper has no learned model: it motivates fast resistance evaluation
with TSV placement and design-option exploration (Sec. I, Sec. IV-B), where
many plans of one stack are compared.  The network is this library's
design, so parity here means "the GPU implements the documented network";
the pins in tests/test_surrogate_cpu.py tie this reference to brute-force
loop definitions of each layer type, to a loop-written forward pass of the
whole network as include/reff_surrogate.h documents it (which fails if the
concatenation order, a pooling step or a skip tensor is wrong), and to
finite differences of its own gradient.  Parity unpinned: none.

Network (C base channels, nt tiers, input 2 nt + 2 channels):
  e1 = 2 x (3x3 conv + ReLU) to C      at full resolution
  e2 = 2 x (3x3 conv + ReLU) to 2C     after 2x2 max pooling
  e3 = 2 x (3x3 conv + ReLU) to 4C     after pooling
  b  = 2 x (3x3 conv + ReLU) to 8C     after pooling
  d3 = 2 x (3x3 conv + ReLU) to 4C of concat(up(b) [4C], e3)
  d2 = 2 x (3x3 conv + ReLU) to 2C of concat(up(d3) [2C], e2)
  d1 = 2 x (3x3 conv + ReLU) to C  of concat(up(d2) [C], e1)
  out = 1x1 conv to nt channels: log R of node (t, x, y)
where up is a 2x2 stride-2 transposed convolution with one bias per
(output offset, channel).
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

LAYERS = ["e1a", "e1b", "e2a", "e2b", "e3a", "e3b", "b1", "b2", "u3", "d3a", "d3b", "u2",
          "d2a", "d2b", "u1", "d1a", "d1b", "head"]


def layer_specs(nt: int, C: int):
    """(name, kind, Cin, Cout, K) in parameter order; kind 'conv' or 'up'."""
    c0 = 2 * nt + 2
    return [
        ("e1a", "conv", c0, C, 3), ("e1b", "conv", C, C, 3),
        ("e2a", "conv", C, 2 * C, 3), ("e2b", "conv", 2 * C, 2 * C, 3),
        ("e3a", "conv", 2 * C, 4 * C, 3), ("e3b", "conv", 4 * C, 4 * C, 3),
        ("b1", "conv", 4 * C, 8 * C, 3), ("b2", "conv", 8 * C, 8 * C, 3),
        ("u3", "up", 8 * C, 4 * C, 1),
        ("d3a", "conv", 8 * C, 4 * C, 3), ("d3b", "conv", 4 * C, 4 * C, 3),
        ("u2", "up", 4 * C, 2 * C, 1),
        ("d2a", "conv", 4 * C, 2 * C, 3), ("d2b", "conv", 2 * C, 2 * C, 3),
        ("u1", "up", 2 * C, C, 1),
        ("d1a", "conv", 2 * C, C, 3), ("d1b", "conv", C, C, 3),
        ("head", "conv", C, nt, 1),
    ]


def num_params(nt: int, C: int) -> int:
    n = 0
    for _, kind, ci, co, k in layer_specs(nt, C):
        g = 4 * co if kind == "up" else co
        n += k * k * ci * g + g
    return n


def _as_t(a):
    return a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a, dtype=np.float64))


def conv_layer(x, w_flat, b, cin: int, cout: int, k: int, relu: bool):
    """K x K convolution (zero padding (K-1)/2) with the stored layout
    W[(kh*K + kw)*Cin + ci][co]: output (x, y) reads input
    (x + kw - (K-1)/2, y + kh - (K-1)/2).  x: [B][Cin][H][W]."""
    w = _as_t(w_flat).reshape(k, k, cin, cout).permute(3, 2, 0, 1)
    y = F.conv2d(x, w, _as_t(b), padding=(k - 1) // 2)
    return F.relu(y) if relu else y


def up_layer(x, w_flat, b_flat, cin: int, cout: int):
    """2x2 stride-2 transposed convolution with the stored layout
    W[ci][(a*2 + c)*Cout + co], bias b[(a*2 + c)*Cout + co], for output pixel
    (2x + c, 2y + a).  x: [B][Cin][H][W] -> [B][Cout][2H][2W]."""
    w = _as_t(w_flat).reshape(cin, 2, 2, cout).permute(0, 3, 1, 2)  # [Cin][Cout][a][c]
    y = F.conv_transpose2d(x, w, stride=2)
    bias = _as_t(b_flat).reshape(2, 2, cout).permute(2, 0, 1)  # [Cout][a][c]
    return y + bias.repeat(1, x.shape[2], x.shape[3]).unsqueeze(0)


def split(params, nt: int, C: int):
    """Flat parameter vector -> {name: (W flat, b flat)} in layer order."""
    p = _as_t(params)
    out = {}
    off = 0
    for name, kind, ci, co, k in layer_specs(nt, C):
        g = 4 * co if kind == "up" else co
        n = k * k * ci * g
        out[name] = (p[off:off + n], p[off + n:off + n + g])
        off += n + g
    assert off == p.numel(), "parameter vector length does not match the architecture"
    return out


def weight_mask(nt: int, C: int) -> np.ndarray:
    """True on the weight entries of the flat vector (False on biases)."""
    m = []
    for _, kind, ci, co, k in layer_specs(nt, C):
        g = 4 * co if kind == "up" else co
        m += [True] * (k * k * ci * g) + [False] * g
    return np.array(m)


def features(desc, nt: int, nx: int, ny: int) -> np.ndarray:
    """Input channels [2 nt + 2][ny][nx]: log gx per tier (0 on the last
    column), log gy per tier (0 on the last row), TSV mask times
    log(1 + mean segment conductance), pad mask."""
    f = np.zeros((2 * nt + 2, ny, nx))
    gx = np.asarray(desc["gx"], dtype=np.float64).reshape(nt, ny, nx - 1)
    gy = np.asarray(desc["gy"], dtype=np.float64).reshape(nt, ny - 1, nx)
    for t in range(nt):
        f[t, :, : nx - 1] = np.log(gx[t])
        f[nt + t, : ny - 1, :] = np.log(gy[t])
    txy = np.asarray(desc["tsv_xy"], dtype=np.int64).reshape(-1, 2)
    tg = np.asarray(desc["tsv_g"], dtype=np.float64).reshape(len(txy), max(nt - 1, 0))
    for j, (x, y) in enumerate(txy):
        mean = tg[j].mean() if nt > 1 else 0.0
        f[2 * nt, y, x] = np.log1p(mean)
    for x, y in np.asarray(desc["pad_xy"], dtype=np.int64).reshape(-1, 2):
        f[2 * nt + 1, y, x] = 1.0
    return f


def bf16_round(a) -> np.ndarray:
    """Round float values to the nearest bfloat16 (ties to even), returned as
    float64: the precision in which the GPU model receives its inputs and
    weights."""
    t = torch.as_tensor(np.asarray(a, dtype=np.float32))
    return t.to(torch.bfloat16).to(torch.float64).numpy()


class _RoundBF16(torch.autograd.Function):
    """Round to bfloat16 in the forward pass (fwd=True) and round the
    incoming gradient in the backward pass: a tensor the GPU model stores in
    bfloat16, together with the gradient it stores for that tensor."""

    @staticmethod
    def forward(ctx, x, fwd):
        return x.to(torch.bfloat16).to(x.dtype) if fwd else x.clone()

    @staticmethod
    def backward(ctx, g):
        return g.to(torch.bfloat16).to(g.dtype), None


def forward(params, x, nt: int, C: int, emulate_bf16: bool = False):
    """x: float64 tensor [B][2nt+2][ny][nx] -> log R prediction [B][nt][ny][nx].

    With emulate_bf16 every tensor the GPU model keeps in bfloat16 is
    rounded where the GPU rounds it: layer outputs (after the ReLU), the
    transposed-convolution outputs, and the gradients with respect to those
    tensors, to each concatenation and to the prediction (which itself stays
    float32 on the GPU).  Sums of gradients arriving at one tensor are
    rounded once, after the sum, as the GPU adds them."""
    P = split(params, nt, C)
    spec = {name: (ci, co, k) for name, _, ci, co, k in layer_specs(nt, C)}

    def q(t, fwd=True):
        return _RoundBF16.apply(t, fwd) if emulate_bf16 else t

    def conv(name, h, relu=True):
        ci, co, k = spec[name]
        return q(conv_layer(h, P[name][0], P[name][1], ci, co, k, relu))

    def up(name, h):
        ci, co, _ = spec[name]
        return q(up_layer(h, P[name][0], P[name][1], ci, co))

    def pool(h):
        return q(F.max_pool2d(h, 2), fwd=False)

    def cat(a, b):
        return q(torch.cat([a, b], dim=1), fwd=False)

    e1 = conv("e1b", conv("e1a", x))
    e2 = conv("e2b", conv("e2a", pool(e1)))
    e3 = conv("e3b", conv("e3a", pool(e2)))
    bt = conv("b2", conv("b1", pool(e3)))
    d3 = conv("d3b", conv("d3a", cat(up("u3", bt), e3)))
    d2 = conv("d2b", conv("d2a", cat(up("u2", d3), e2)))
    d1 = conv("d1b", conv("d1a", cat(up("u1", d2), e1)))
    ci, co, k = spec["head"]
    out = conv_layer(d1, P["head"][0], P["head"][1], ci, co, k, False)
    return q(out, fwd=False)


def masked_loss(pred, labels, nt: int, nx: int, ny: int, pad_masks):
    """Mean of (pred - log R)^2 over the labelled non-pad nodes (a node listed
    twice counts once, with its first value).  labels: per plan (node ids,
    R values); pad_masks: per plan [ny][nx] booleans."""
    terms = []
    for b, (nodes, R) in enumerate(labels):
        seen = set()
        for v, r in zip(np.asarray(nodes).tolist(), np.asarray(R).tolist()):
            t, rem = divmod(int(v), nx * ny)
            y, x = divmod(rem, nx)
            if (t == 0 and pad_masks[b][y, x]) or v in seen:
                continue
            seen.add(v)
            terms.append(pred[b, t, y, x] - float(np.log(r)))
    if not terms:
        return pred.sum() * 0.0
    d = torch.stack(terms)
    return (d * d).mean()


def loss_and_grad(params, descs, labels, nt: int, nx: int, ny: int, C: int,
                  quantise_inputs: bool = True, emulate_bf16: bool = False):
    """Reference loss and gradient with respect to the flat parameter vector.
    With quantise_inputs the weights and input channels are first rounded
    to bfloat16, as the GPU model receives them; emulate_bf16 see forward."""
    p = np.asarray(params, dtype=np.float64)
    feats = np.stack([features(d, nt, nx, ny) for d in descs])
    if quantise_inputs:
        # weights and input channels reach the matrix cores as bfloat16;
        # biases stay float32
        m = weight_mask(nt, C)
        p = np.where(m, bf16_round(p), p)
        feats = bf16_round(feats)
    pt = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    x = torch.as_tensor(feats)
    pads = [features(d, nt, nx, ny)[2 * nt + 1] > 0 for d in descs]
    pred = forward(pt, x, nt, C, emulate_bf16=emulate_bf16)
    loss = masked_loss(pred, labels, nt, nx, ny, pads)
    loss.backward()
    return loss.item(), pt.grad.numpy().copy(), pred.detach().numpy()
