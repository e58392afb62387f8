"""Seeded synthetic inputs (wave-number fields, sources, batch draws).

This module holds no part of the solver's arithmetic: it only produces the
problem data (element-wise wave numbers, source positions, problem sizes) in
the shapes of the paper's model problems, so that the GPU library and the CPU
oracle are fed the very same arrays.

Randomness comes from SplitMix64 (Steele, Lea, Flood 2014: state += golden
gamma; two xor-shift-multiply rounds) turned into uniforms in [0, 1) by the
top 53 bits, and into normals by Box-Muller.
"""
import math

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n):
    """n consecutive SplitMix64 outputs for the given 64-bit seed (uint64 array)."""
    with np.errstate(over="ignore"):
        s = np.uint64(seed) + _GAMMA * np.arange(1, n + 1, dtype=np.uint64)
        z = s
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniforms(seed, n):
    """n uniforms in [0, 1) from the top 53 bits of SplitMix64."""
    return (splitmix64(seed, n) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normals(seed, n):
    """n standard normals by Box-Muller from 2*ceil(n/2) uniforms."""
    m = (n + 1) // 2
    u = uniforms(seed, 2 * m)
    u1 = 1.0 - u[0::2]                     # (0, 1]
    u2 = u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.concatenate([r * np.cos(2 * np.pi * u2), r * np.sin(2 * np.pi * u2)])
    return z[:n]


def element_centroids(n_el):
    """Centroid coordinate of each of the n_el uniform elements on [0, 1]."""
    return (np.arange(n_el) + 0.5) / n_el


def wedge_k(n_el, k0):
    """Three-layer wedge wave number, sampled at the centroids of n_el x n_el elements.

    Layers split by the lines y = 0.6 + 0.2 x and y = 0.3 - 0.1 x: k0 above the
    upper line (a point on a line belongs to the upper region), 1.5 k0 between
    them and 2 k0 below.  Returns k (not k^2), shape (n_el, n_el), x fastest.
    """
    c = element_centroids(n_el)
    x = c[None, :]
    y = c[:, None]
    k = np.where(y >= 0.6 + 0.2 * x, k0, np.where(y >= 0.3 - 0.1 * x, 1.5 * k0, 2.0 * k0))
    return np.ascontiguousarray(k, dtype=np.float64)


def gaussian_random_field(n_el, corr_len=0.1, seed=0):
    """Unit-variance Gaussian random field with squared-exponential covariance.

    C(r) = exp(-r^2 / (2 l^2)), sampled at the n_el x n_el element centroids of
    the unit square by circulant embedding on a periodic 2n_el x 2n_el grid of
    spacing 1/n_el (eigenvalues clipped at zero), driven by SplitMix64 normals.
    Returns g clipped to [-1, 1], shape (n_el, n_el), x fastest.
    """
    m = 2 * n_el
    d = np.minimum(np.arange(m), m - np.arange(m)) / n_el
    r2 = d[None, :] ** 2 + d[:, None] ** 2
    cov = np.exp(-r2 / (2.0 * corr_len ** 2))
    lam = np.maximum(np.real(np.fft.fft2(cov)), 0.0)
    z = normals(seed, 2 * m * m).reshape(2, m, m)
    w = np.fft.fft2(np.sqrt(lam / (m * m)) * (z[0] + 1j * z[1]))
    g = np.real(w)[:n_el, :n_el]
    return np.ascontiguousarray(np.clip(g, -1.0, 1.0))


def grf_k(n_el, kbar=300.0, amp=0.3, corr_len=0.1, seed=0):
    """Heterogeneous wave number k = kbar (1 + amp g), g the clipped random field above."""
    return kbar * (1.0 + amp * gaussian_random_field(n_el, corr_len, seed))


def batch_draws(n=64, seed=0, k_lo=50.0, k_hi=400.0, kh=0.625, degrees=(2, 3, 4)):
    """Problem list for batched solves: k ~ U[k_lo, k_hi], p ~ U(degrees), source ~ U(0,1)^2.

    Elements per side = ceil(k / kh).  Draw order per problem: k, p, x0, y0.
    """
    u = uniforms(seed, 4 * n).reshape(n, 4)
    out = []
    for i in range(n):
        k = k_lo + (k_hi - k_lo) * u[i, 0]
        p = degrees[min(int(u[i, 1] * len(degrees)), len(degrees) - 1)]
        out.append({"k": float(k), "p": int(p), "n_el": int(math.ceil(k / kh)),
                    "x0": (float(u[i, 2]), float(u[i, 3]))})
    return out


# The five workloads (shapes of the paper's model problems MP 1-B, MP 2-A, MP 2-B).
CONFIGS = {
    "c0_1d_k50_p2": dict(dim=1, p=2, n_el=80, k=50.0, x0=(0.5,), defl_mode=1),
    "c1_2d_k100_p3": dict(dim=2, p=3, n_el=160, k=100.0, x0=(0.5, 0.5), defl_mode=2),
    "c2_wedge_k150": dict(dim=2, p=3, n_el=480, k0=150.0, x0=(0.5, 0.95), defl_mode=2),
    "c4_grf_k300_p4": dict(dim=2, p=4, n_el=960, kbar=300.0, x0=(0.5, 0.5), defl_mode=2),
}
