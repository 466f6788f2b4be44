"""Pins of the screening model's CPU reference (oracle/surrogate_ref.py) and
host-side checks of its C ABI that need no GPU.

The reference is pinned to things other than itself: each layer type
against a brute-force loop written from the layout that
include/reff_surrogate.h documents, the input channels against values
worked out by hand, and the autograd gradient against central finite
differences."""
import ctypes as C

import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import surrogate_ref as sr
from paper_2607_05818_amd import gen


def test_conv_layer_matches_loop_definition():
    rng = np.random.default_rng(3)
    for k in (3, 1):
        cin, cout, H, W = 3, 4, 5, 6
        w = rng.normal(size=k * k * cin * cout)
        b = rng.normal(size=cout)
        x = rng.normal(size=(2, cin, H, W))
        got = sr.conv_layer(torch.as_tensor(x), w, b, cin, cout, k, relu=False).numpy()
        h = (k - 1) // 2
        want = np.zeros((2, cout, H, W))
        for n in range(2):
            for co in range(cout):
                for y in range(H):
                    for xx in range(W):
                        s = b[co]
                        for kh in range(k):
                            for kw in range(k):
                                sy, sx = y + kh - h, xx + kw - h
                                if 0 <= sy < H and 0 <= sx < W:
                                    for ci in range(cin):
                                        s += w[((kh * k + kw) * cin + ci) * cout + co] * x[n, ci, sy, sx]
                        want[n, co, y, xx] = s
        assert np.allclose(got, want, rtol=1e-12, atol=1e-12)
        relu = sr.conv_layer(torch.as_tensor(x), w, b, cin, cout, k, relu=True).numpy()
        assert np.array_equal(relu, np.maximum(got, 0.0))


def test_up_layer_matches_loop_definition():
    rng = np.random.default_rng(4)
    cin, cout, H, W = 3, 2, 3, 4
    w = rng.normal(size=cin * 4 * cout)
    b = rng.normal(size=4 * cout)
    x = rng.normal(size=(1, cin, H, W))
    got = sr.up_layer(torch.as_tensor(x), w, b, cin, cout).numpy()
    want = np.zeros((1, cout, 2 * H, 2 * W))
    for co in range(cout):
        for y in range(H):
            for xx in range(W):
                for a in range(2):
                    for c in range(2):
                        s = b[(a * 2 + c) * cout + co]
                        for ci in range(cin):
                            s += w[ci * 4 * cout + (a * 2 + c) * cout + co] * x[0, ci, y, xx]
                        want[0, co, 2 * y + a, 2 * xx + c] = s
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12)


def test_feature_channels_by_hand():
    nt, nx, ny = 2, 3, 2
    gx = np.arange(1, 1 + nt * ny * (nx - 1), dtype=float).reshape(nt, ny, nx - 1)
    gy = np.arange(1, 1 + nt * (ny - 1) * nx, dtype=float).reshape(nt, ny - 1, nx) * 2
    d = gen.make_desc(nt, nx, ny, gx, gy, [(2, 1)], [[3.0]], [(0, 0), (1, 1)])
    f = sr.features(d, nt, nx, ny)
    assert f.shape == (6, 2, 3)
    # log gx of tier 1 at (x=1, y=1): edge (1,1)-(2,1) = gx[1][1][1] = 8
    assert f[1, 1, 1] == pytest.approx(np.log(8.0))
    assert f[0, 0, 2] == 0.0 and f[1, 1, 2] == 0.0  # last column
    # log gy of tier 0 at (x=2, y=0): edge (2,0)-(2,1) = gy[0][0][2] = 6
    assert f[2, 0, 2] == pytest.approx(np.log(6.0))
    assert np.all(f[2:4, 1, :] == 0.0)  # last row
    assert f[4, 1, 2] == pytest.approx(np.log(4.0)) and f[4].sum() == pytest.approx(np.log(4.0))
    assert f[5, 0, 0] == 1.0 and f[5, 1, 1] == 1.0 and f[5].sum() == 2.0


def test_parameter_layout_consumes_vector():
    for nt, C in ((3, 32), (2, 4)):
        n = sr.num_params(nt, C)
        assert len(sr.weight_mask(nt, C)) == n
        parts = sr.split(np.zeros(n), nt, C)
        assert list(parts) == sr.LAYERS
    with pytest.raises(AssertionError):
        sr.split(np.zeros(sr.num_params(2, 4) + 1), 2, 4)


def test_reference_gradient_matches_finite_differences():
    """Autograd gradient of the masked log-R loss against central
    differences, at coordinates in every layer (float64, no rounding)."""
    nt, nx, ny, C = 2, 8, 8, 4
    descs = [gen.small_random_desc(40 + i, nt, nx, ny, 5, 2) for i in range(2)]
    rng = np.random.default_rng(7)
    n = sr.num_params(nt, C)
    p = rng.normal(scale=0.3, size=n)
    labels = [(rng.choice(nt * nx * ny, size=20, replace=False),
               rng.uniform(0.2, 3.0, size=20)) for _ in descs]
    _, g, _ = sr.loss_and_grad(p, descs, labels, nt, nx, ny, C, quantise_inputs=False)

    def loss_at(q):
        return sr.loss_and_grad(q, descs, labels, nt, nx, ny, C, quantise_inputs=False)[0]

    offs = np.cumsum([0] + [len(w) + len(b) for w, b in sr.split(p, nt, C).values()])
    idx = []
    for a, b in zip(offs[:-1], offs[1:]):
        idx += list(rng.integers(a, b, size=2))
    h = 1e-6
    for i in idx:
        e = np.zeros(n)
        e[i] = h
        fd = (loss_at(p + e) - loss_at(p - e)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(fd)), (i, fd, g[i])


# --- the network's composition, written with loops from the header ---------

def _loop_conv(x, w, b, cin, cout, k, relu):
    """x[Cin][H][W]; header layout W[(kh*K + kw)*Cin + ci][Cout]; output
    (x, y) reads input (x + kw - (K-1)/2, y + kh - (K-1)/2), zero outside."""
    _, H, W = x.shape
    h = (k - 1) // 2
    out = np.zeros((cout, H, W))
    for co in range(cout):
        for yy in range(H):
            for xx in range(W):
                s = b[co]
                for kh in range(k):
                    for kw in range(k):
                        sy, sx = yy + kh - h, xx + kw - h
                        if 0 <= sy < H and 0 <= sx < W:
                            for ci in range(cin):
                                s += w[((kh * k + kw) * cin + ci) * cout + co] * x[ci, sy, sx]
                out[co, yy, xx] = max(s, 0.0) if relu else s
    return out


def _loop_pool(x):
    c, H, W = x.shape
    out = np.zeros((c, H // 2, W // 2))
    for ch in range(c):
        for yy in range(H // 2):
            for xx in range(W // 2):
                out[ch, yy, xx] = max(x[ch, 2 * yy, 2 * xx], x[ch, 2 * yy, 2 * xx + 1],
                                      x[ch, 2 * yy + 1, 2 * xx], x[ch, 2 * yy + 1, 2 * xx + 1])
    return out


def _loop_up(x, w, b, cin, cout):
    """Header layout W[ci][(a*2 + b)*Cout + co], bias [(a*2 + b)*Cout + co],
    output pixel (2x + b, 2y + a)."""
    _, H, W = x.shape
    out = np.zeros((cout, 2 * H, 2 * W))
    for co in range(cout):
        for yy in range(H):
            for xx in range(W):
                for a in range(2):
                    for c in range(2):
                        s = b[(a * 2 + c) * cout + co]
                        for ci in range(cin):
                            s += w[ci * 4 * cout + (a * 2 + c) * cout + co] * x[ci, yy, xx]
                        out[co, 2 * yy + a, 2 * xx + c] = s
    return out


def _loop_network(p, x, nt, C, variant=None):
    """The network as include/reff_surrogate.h documents it, one plan
    x[2nt+2][ny][nx] -> [nt][ny][nx].  variant plants one mistake."""
    cin0 = 2 * nt + 2
    convs = [("e1a", cin0, C), ("e1b", C, C), ("e2a", C, 2 * C), ("e2b", 2 * C, 2 * C),
             ("e3a", 2 * C, 4 * C), ("e3b", 4 * C, 4 * C), ("b1", 4 * C, 8 * C),
             ("b2", 8 * C, 8 * C), ("u3", 8 * C, 4 * C), ("d3a", 8 * C, 4 * C),
             ("d3b", 4 * C, 4 * C), ("u2", 4 * C, 2 * C), ("d2a", 4 * C, 2 * C),
             ("d2b", 2 * C, 2 * C), ("u1", 2 * C, C), ("d1a", 2 * C, C), ("d1b", C, C),
             ("head", C, nt)]
    P, off = {}, 0
    for name, ci, co in convs:
        if name.startswith("u"):
            nw, nb = ci * 4 * co, 4 * co
        else:
            k = 1 if name == "head" else 3
            nw, nb = k * k * ci * co, co
        P[name] = (p[off:off + nw], p[off + nw:off + nw + nb], ci, co)
        off += nw + nb
    assert off == len(p)

    def conv(name, h, relu=True):
        w, b, ci, co = P[name]
        return _loop_conv(h, w, b, ci, co, 1 if name == "head" else 3, relu)

    def up(name, h):
        w, b, ci, co = P[name]
        return _loop_up(h, w, b, ci, co)

    def cat(u, e):
        return np.concatenate([e, u] if variant == "concat_swapped" else [u, e])

    e1 = conv("e1b", conv("e1a", x))
    if variant == "pool_between_convs":
        e2 = conv("e2b", _loop_pool(conv("e2a", e1)))
    else:
        e2 = conv("e2b", conv("e2a", _loop_pool(e1)))
    e3 = conv("e3b", conv("e3a", _loop_pool(e2)))
    bt = conv("b2", conv("b1", _loop_pool(e3)))
    d3 = conv("d3b", conv("d3a", cat(up("u3", bt), e3)))
    d2 = conv("d2b", conv("d2a", cat(up("u2", d3), e2)))
    skip1 = e1 if variant != "skip_from_first_conv" else conv("e1a", x)
    d1 = conv("d1b", conv("d1a", cat(up("u1", d2), skip1)))
    return conv("head", d1, relu=False)


def test_network_composition_matches_loop_definition():
    """forward() against the network written out with loops from the
    header's documentation (nt = 1, C = 2, 8 x 8, float64), and each of
    three plausible composition mistakes (concatenation order, a pooling
    step in the wrong place, the wrong skip tensor) moves the output far
    beyond the agreement bar."""
    nt, C, H, W = 1, 2, 8, 8
    rng = np.random.default_rng(21)
    n = sr.num_params(nt, C)
    p = rng.normal(scale=0.5, size=n)
    x = rng.normal(size=(2, 2 * nt + 2, H, W))
    got = sr.forward(torch.as_tensor(p), torch.as_tensor(x), nt, C).numpy()
    assert got.shape == (2, nt, H, W)
    for i in range(2):
        want = _loop_network(p, x[i], nt, C)
        assert np.allclose(got[i], want, rtol=1e-11, atol=1e-11)
    for variant in ("concat_swapped", "pool_between_convs", "skip_from_first_conv"):
        bad = _loop_network(p, x[0], nt, C, variant)
        assert np.max(np.abs(bad - got[0])) > 1e-3, variant


def test_loss_counts_labels_once_and_skips_pads():
    nt, nx, ny = 1, 4, 4
    pred = torch.zeros((1, nt, ny, nx), dtype=torch.float64)
    pads = [np.zeros((ny, nx), dtype=bool)]
    pads[0][0, 0] = True
    e = np.e
    loss = sr.masked_loss(pred, [([0, 5, 5, 6], [e, e, e ** 3, e ** 2])], nt, nx, ny, pads)
    # node 0 is a pad; node 5 counts once with log R = 1; node 6 has log R = 2
    assert float(loss) == pytest.approx((1.0 + 4.0) / 2)


@pytest.mark.parametrize("cfg", [(3, 12, 16, 32), (3, 16, 16, 6), (0, 16, 16, 32), (40, 16, 16, 32)])
def test_surrogate_create_rejects_bad_config_on_host(cfg):
    from paper_2607_05818_amd import reff
    with pytest.raises(reff.ReffError) as ei:
        reff.reff_surrogate_create(*cfg)
    assert ei.value.status == reff.REFF_ERR_INVALID_ARG
