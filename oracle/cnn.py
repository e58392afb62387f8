"""Learned smoother network of the CPU oracle (test infrastructure only).

Not in the paper (which keeps damped Jacobi and notes that non-standard
smoothers are outside its scope); this is the oracle of the library's learned
fine-level smoother.  Parity of this module is pinned only by its own
mathematics (finite-difference gradients, a single layer against a library
correlation, the zero-weight case); there is no printed value to pin it to.

Network C: 4 complex 3x3 convolution layers on the interior control-point grid
[n2][n1]; channels 2 -> 16 -> 16 -> 16 -> 1; CReLU (ReLU of the real and the
imaginary part separately) after the first three layers; zero padding.
Input channels: the residual scaled by its root mean square, r/rms(r) with
rms(r) = ||r|| / sqrt(N) (entries of order one whatever the grid size), and the
real feature c = k^2 h^2 (k of the finest element at the control point's
index, clamped).  Smoother step: the damped Jacobi update plus a learned
correction,
    s = omega D^-1 r + rms(r) C(r/rms(r), c),
homogeneous of degree 1 in r; zero weights give exactly damped Jacobi.
Training loss for one residual r: L = ||r - M_beta s||^2 / ||r||^2.

Complex gradients follow the convention g_z = dL/dRe(z) + i dL/dIm(z): for
y = W x, g_x = conj(W) g_y and g_W = g_y conj(x).
"""
import numpy as np

CHANNELS = (2, 16, 16, 16, 1)


def init_params(seed=0, channels=CHANNELS, scale=0.5):
    """Complex weights (Cout, Cin, 3, 3) and biases (Cout,) per layer (seeded)."""
    rng = np.random.default_rng(seed)
    params = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        s = scale / np.sqrt(9 * cin)
        W = s * (rng.standard_normal((cout, cin, 3, 3)) + 1j * rng.standard_normal((cout, cin, 3, 3)))
        b = 0.01 * (rng.standard_normal(cout) + 1j * rng.standard_normal(cout))
        params.append((W, b))
    return params


def conv(x, W, b):
    """y[o, h, w] = b[o] + sum_{i,dy,dx} W[o, i, dy, dx] x[i, h+dy-1, w+dx-1] (zero outside)."""
    cin, H, Wd = x.shape
    xp = np.zeros((cin, H + 2, Wd + 2), dtype=np.complex128)
    xp[:, 1:-1, 1:-1] = x
    y = np.zeros((W.shape[0], H, Wd), dtype=np.complex128) + b[:, None, None]
    for dy in range(3):
        for dx in range(3):
            y += np.einsum("oi,ihw->ohw", W[:, :, dy, dx], xp[:, dy:dy + H, dx:dx + Wd])
    return y


def conv_backward(x, W, gy):
    """Gradients of a conv layer: (g_x, g_W, g_b) for upstream g_y."""
    cin, H, Wd = x.shape
    xp = np.zeros((cin, H + 2, Wd + 2), dtype=np.complex128)
    xp[:, 1:-1, 1:-1] = x
    gW = np.zeros_like(W)
    gxp = np.zeros_like(xp)
    for dy in range(3):
        for dx in range(3):
            gW[:, :, dy, dx] = np.einsum("ohw,ihw->oi", gy, np.conj(xp[:, dy:dy + H, dx:dx + Wd]))
            gxp[:, dy:dy + H, dx:dx + Wd] += np.einsum("oi,ohw->ihw", np.conj(W[:, :, dy, dx]), gy)
    gb = gy.sum(axis=(1, 2))
    return gxp[:, 1:-1, 1:-1], gW, gb


def crelu(z):
    return np.maximum(z.real, 0.0) + 1j * np.maximum(z.imag, 0.0)


def crelu_backward(z, g):
    return g.real * (z.real > 0) + 1j * g.imag * (z.imag > 0)


def forward(params, z, c, keep=False):
    """Network output for input field z (H, W) complex and feature c (H, W) real."""
    x = np.stack([z, c.astype(np.complex128)])
    acts = [x]
    pre = []
    for l, (W, b) in enumerate(params):
        y = conv(x, W, b)
        pre.append(y)
        x = crelu(y) if l + 1 < len(params) else y
        acts.append(x)
    out = x[0]
    return (out, acts, pre) if keep else out


def feature(k2_elem, n_el, n, length=1.0):
    """c[i2, i1] = k^2 h^2 of the finest element (min(i2, n_el-1), min(i1, n_el-1)),
    h = length / n_el the x extent of an element."""
    n2, n1 = n
    h = length / n_el
    i2 = np.minimum(np.arange(n2), k2_elem.shape[0] - 1)
    i1 = np.minimum(np.arange(n1), k2_elem.shape[1] - 1)
    return k2_elem[np.ix_(i2, i1)] * h * h


def smoother_step(params, r, c, shape, D, omega):
    """s = omega D^-1 r + rms(r) C(r/rms(r), c) on the grid `shape` (r flat, x fastest)."""
    rms = np.linalg.norm(r) / np.sqrt(r.size)
    if rms == 0.0:
        return np.zeros_like(r)
    return omega * r / D + rms * forward(params, (r / rms).reshape(shape), c).reshape(-1)


def loss_and_grad(params, r, c, shape, Mb, D, omega):
    """L = ||r - Mb s||^2 / ||r||^2 and its gradients with respect to every W, b."""
    nr = np.linalg.norm(r)
    rms = nr / np.sqrt(r.size)
    out, acts, pre = forward(params, (r / rms).reshape(shape), c, keep=True)
    s = omega * r / D + rms * out.reshape(-1)
    e = r - Mb @ s
    L = np.vdot(e, e).real / nr ** 2
    g_e = 2.0 * e / nr ** 2
    g_s = -(Mb.conj().T @ g_e)
    g = (rms * g_s).reshape(shape)[None]         # gradient w.r.t. the output channel
    grads = [None] * len(params)
    for l in range(len(params) - 1, -1, -1):
        W, b = params[l]
        if l + 1 < len(params):
            g = crelu_backward(pre[l], g)
        gx, gW, gb = conv_backward(acts[l], W, g)
        grads[l] = (gW, gb)
        g = gx
    return L, grads
