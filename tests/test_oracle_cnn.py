"""Pins of the oracle's learned-smoother network: finite differences, a library
correlation, and structural special cases (parity otherwise unpinned: the
network is not in the paper)."""
import numpy as np
import pytest
import scipy.ndimage as ndi

from oracle import cnn
from oracle import helmholtz as hz
from oracle import solver as osv


def _tiny():
    prob = hz.Problem(2, 2, 6, 7.0)
    s = osv.Solver(prob, osv.Options(mg_min_elems=3, defl_mode=0))
    lv = s.levels[0]
    shape = (lv.n[1], lv.n[0])
    c = cnn.feature(np.full((6, 6), 49.0), 6, shape)
    rng = np.random.default_rng(5)
    r = rng.standard_normal(lv.N) + 1j * rng.standard_normal(lv.N)
    return lv.Mb.toarray(), r, c, shape, lv.D, lv.omega


def test_single_layer_is_a_zero_padded_correlation():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((1, 7, 5))
    W = rng.standard_normal((1, 1, 3, 3))
    y = cnn.conv(x.astype(complex), W.astype(complex), np.zeros(1, complex))
    ref = ndi.correlate(x[0], W[0, 0], mode="constant", cval=0.0)
    assert np.allclose(y[0].real, ref, atol=1e-13) and np.allclose(y[0].imag, 0)


def test_zero_weights_give_damped_jacobi():
    Mb, r, c, shape, D, w = _tiny()
    params = [(np.zeros_like(W), np.zeros_like(b)) for W, b in cnn.init_params(1)]
    s = cnn.smoother_step(params, r, c, shape, D, w)
    assert np.array_equal(s, w * r / D)
    L, _ = cnn.loss_and_grad(params, r, c, shape, Mb, D, w)
    ej = r - Mb @ (w * r / D)
    assert abs(L - np.vdot(ej, ej).real / np.vdot(r, r).real) < 1e-13


def test_step_is_homogeneous_of_degree_one():
    Mb, r, c, shape, D, w = _tiny()
    params = cnn.init_params(2)
    a = cnn.smoother_step(params, 3.5 * r, c, shape, D, w)
    b = 3.5 * cnn.smoother_step(params, r, c, shape, D, w)
    assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(b).max())


@pytest.mark.parametrize("layer", [0, 1, 3])
def test_gradients_match_finite_differences(layer):
    Mb, r, c, shape, D, w = _tiny()
    params = cnn.init_params(3, scale=1.0)
    L, grads = cnn.loss_and_grad(params, r, c, shape, Mb, D, w)
    rng = np.random.default_rng(layer)
    W, b = params[layer]
    gW, gb = grads[layer]
    h = 1e-6
    for _ in range(6):
        idx = tuple(rng.integers(0, s) for s in W.shape)
        for part, unit in (("re", 1.0), ("im", 1j)):
            def loss_with(delta):
                P = [(Wl.copy(), bl.copy()) for Wl, bl in params]
                P[layer][0][idx] += delta * unit
                return cnn.loss_and_grad(P, r, c, shape, Mb, D, w)[0]
            fd = (loss_with(h) - loss_with(-h)) / (2 * h)
            an = gW[idx].real if part == "re" else gW[idx].imag
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (layer, idx, part, fd, an)
    # a bias entry
    o = 0
    def loss_b(delta):
        P = [(Wl.copy(), bl.copy()) for Wl, bl in params]
        P[layer][1][o] += delta
        return cnn.loss_and_grad(P, r, c, shape, Mb, D, w)[0]
    fd = (loss_b(h) - loss_b(-h)) / (2 * h)
    assert abs(fd - gb[o].real) <= 1e-6 * max(1.0, abs(fd))
