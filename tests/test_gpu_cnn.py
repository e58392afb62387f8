"""Learned finest-level smoother on the GPU against the oracle network.

The library evaluates the network with BF16 activations and weights and FP32
accumulation; the oracle runs the same network in FP64 from the same FP32
parameters.  BF16 keeps 8 significant bits (unit roundoff 2^-9); four layers
of 3x3x32 dot products with rounding of every input give a relative error of
a few 1e-3 on the network output, and the gradient inherits that plus the rare
CReLU mask flips at pre-activations within that error of zero.  The bars:
loss within 2e-2 relative, gradient within 5e-2 relative in norm with cosine
similarity above 0.995, and one V-cycle within 1e-2 of the oracle's relative
to the network's share of it.  With zero weights the learned smoother is
exactly damped Jacobi, which the FP64 path reproduces to 1e-12.
"""
import sys

import numpy as np
import pytest

from oracle import cnn as ocnn
from oracle import helmholtz as hz
from oracle import solver as osv
from paper_2010_10232_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.complex128)).to("cuda")


def to_host(t):
    return t.cpu().numpy()


def rel(a, b):
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def flat(params):
    """Oracle parameters -> the library's vector: per layer W[o][i][dy][dx] then b, (re, im) floats."""
    z = np.concatenate([np.concatenate([Wt.reshape(-1), b]) for Wt, b in params])
    return np.stack([z.real, z.imag], -1).reshape(-1).astype(np.float32)


def unflat(v, like):
    z = v[0::2].astype(np.float64) + 1j * v[1::2].astype(np.float64)
    out, o = [], 0
    for Wt, b in like:
        nw = Wt.size
        out.append((z[o:o + nw].reshape(Wt.shape), z[o + nw:o + nw + b.size]))
        o += nw + b.size
    return out


def f32_params(seed, scale):
    """Seeded oracle parameters rounded to FP32 (the library's master precision)."""
    return unflat(flat(ocnn.init_params(seed, scale=scale)), ocnn.init_params(seed))


CASES = {
    "2d_p3_k40_101": dict(dim=2, p=3, n_el=100, k=40.0),
    "2d_grf_p2_90": dict(dim=2, p=2, n_el=90, grf=30.0),
    "1d_p2_k60_300": dict(dim=1, p=2, n_el=300, k=60.0),
}


def _k_field(c):
    return W.grf_k(c["n_el"], kbar=c["grf"], seed=2) if "grf" in c else None


_cache = {}


def build(name):
    if name in _cache:
        return _cache[name]
    from paper_2010_10232_amd import binding as B
    c = CASES[name]
    ke = _k_field(c)
    k = c.get("k", 1.0)
    _say(f"[cnn case {name}] oracle + gpu setup")
    op = hz.Problem(c["dim"], c["p"], c["n_el"], k, k_elem=ke)
    osol = osv.Solver(op, osv.Options(defl_mode=1))
    gp = B.Problem(c["dim"], c["p"], c["n_el"], k=k, k_elem=ke)
    gs = B.Solver(gp, defl_mode=1)
    _cache[name] = (c, op, osol, gp, gs)
    return _cache[name]


def _shape(osol, op):
    lv = osol.levels[0]
    return (lv.n[1], lv.n[0]) if op.dim == 2 else (1, lv.n[0])


def test_params_roundtrip_and_reject():
    from paper_2010_10232_amd import binding as B
    net = B.Cnn(seed=3)
    ref = ocnn.init_params(0)
    assert net.n_floats == 2 * sum(Wt.size + b.size for Wt, b in ref)
    v = flat(f32_params(5, 0.5))
    net.set_params(v)
    assert np.array_equal(net.get_params(), v)
    bad = v.copy()
    bad[7] = np.nan
    with pytest.raises(Exception):
        net.set_params(bad)
    assert np.array_equal(net.get_params(), v)


@pytest.mark.parametrize("name", list(CASES))
def test_loss_and_gradient_vs_oracle(name):
    from paper_2010_10232_amd import binding as B
    c, op, osol, gp, gs = build(name)
    params = f32_params(11, 0.5)
    net = B.Cnn()
    net.set_params(flat(params))
    lv = osol.levels[0]
    rng = np.random.default_rng(21)
    r = rng.standard_normal(lv.N) + 1j * rng.standard_normal(lv.N)
    _say(f"[cnn case {name}] loss/grad N={lv.N}")
    L_gpu, g_gpu = net.loss_grad(gs, to_dev(r))
    L_ref, grads = ocnn.loss_and_grad(params, r, osol.cnn_feature(), _shape(osol, op), lv.Mb, lv.D, lv.omega)
    g_ref = flat([(gW, gb) for gW, gb in grads]).astype(np.float64)
    _say(f"  loss gpu {L_gpu:.6e} oracle {L_ref:.6e}")
    assert abs(L_gpu - L_ref) <= 2e-2 * L_ref
    g = g_gpu.astype(np.float64)
    e = rel(g, g_ref)
    cos = float(g @ g_ref / (np.linalg.norm(g) * np.linalg.norm(g_ref)))
    _say(f"  grad rel {e:.3e} cos {cos:.6f}")
    assert e <= 5e-2 and cos >= 0.995


@pytest.mark.parametrize("name", list(CASES))
def test_zero_weights_are_damped_jacobi(name):
    from paper_2010_10232_amd import binding as B
    c, op, osol, gp, gs = build(name)
    N = osol.levels[0].N
    x = np.random.default_rng(4).standard_normal(N) + 0j
    ref = to_host(gs.apply("VCYCLE", 0, to_dev(x)))
    net = B.Cnn()
    net.set_params(np.zeros(net.n_floats, dtype=np.float32))
    gs.set_smoother(net)
    try:
        got = to_host(gs.apply("VCYCLE", 0, to_dev(x)))
    finally:
        gs.set_smoother(None)
    e = rel(got, ref)
    _say(f"[cnn case {name}] zero-weight V-cycle vs Jacobi {e:.2e}")
    assert e <= 1e-12
    assert rel(got, osol.vcycle(0, x)) <= 1e-11


@pytest.mark.parametrize("name", list(CASES))
def test_learned_vcycle_vs_oracle(name):
    from paper_2010_10232_amd import binding as B
    c, op, osol, gp, gs = build(name)
    params = f32_params(13, 0.1)
    net = B.Cnn()
    net.set_params(flat(params))
    N = osol.levels[0].N
    x = np.random.default_rng(6).standard_normal(N) + 1j * np.random.default_rng(7).standard_normal(N)
    gs.set_smoother(net)
    try:
        got = to_host(gs.apply("VCYCLE", 0, to_dev(x)))
    finally:
        gs.set_smoother(None)
    lsol = osv.Solver(op, osv.Options(defl_mode=1), cnn_params=params)
    ref = lsol.vcycle(0, x)
    jac = osol.vcycle(0, x)
    share = np.linalg.norm(ref - jac)
    e = float(np.linalg.norm(got - ref) / share)
    _say(f"[cnn case {name}] learned V-cycle: error / network share {e:.3e} (share {share / np.linalg.norm(ref):.3e})")
    assert share > 1e-3 * np.linalg.norm(ref)
    assert e <= 1e-2


def test_capture_train_and_solve(tmp_path):
    """Capture, training in the library (hh_cnn_train, weights also written to a
    file), then the learned smoother in the mixed form: the solve converges, takes
    no more iterations than with Jacobi, and at tol 1e-10 stays within 1e-6 of the
    oracle's FP64 solution (the mixed-precision bar)."""
    from paper_2010_10232_amd import binding as B
    import torch
    c, op, osol, gp, gs = build("2d_grf_p2_90")
    N = osol.levels[0].N
    f = gp.point_source((0.5, 0.5))
    buf = torch.zeros((16, N), dtype=torch.complex128, device="cuda")
    gs.capture(buf, 16)
    u, info_j = gs.solve(f)
    gs.capture(None, 0)
    n = gs.captured()
    _say(f"[cnn train] captured {n} samples, Jacobi its {info_j['iters']}")
    assert 4 <= n <= 16
    samples = buf[:n]
    assert torch.isfinite(torch.view_as_real(samples)).all()
    net = B.Cnn()
    net.set_params(flat(f32_params(17, 0.05)))
    L0 = np.mean([net.loss_grad(gs, samples[i])[0] for i in range(n)])
    wpath = tmp_path / "net.hhw"
    l0, l1 = net.train([gs], [samples], steps=200, lr=2e-3, seed=0, out_weights=str(wpath))
    _say(f"[cnn train] mean loss {l0:.4e} -> {l1:.4e}")
    assert abs(l0 - L0) <= 1e-9 * L0 and l1 < 0.9 * l0
    assert np.array_equal(B.Cnn(path=str(wpath)).get_params(), net.get_params())
    gs.set_smoother(net)
    try:
        u2, info_l = gs.solve(f)
    finally:
        gs.set_smoother(None)
    _say(f"[cnn train] learned-smoother solve its {info_l['iters']} (Jacobi {info_j['iters']})")
    assert info_l["converged"] and info_l["iters"] <= info_j["iters"]
    A = osol.levels[0].A
    fh, uh = to_host(f), to_host(u2)
    assert np.linalg.norm(fh - A @ uh) <= 1.01e-7 * np.linalg.norm(fh)
    # mixed form (FP32 V-cycle) with the network against the oracle's FP64 solution, tol 1e-10
    g32 = B.Solver(gp, defl_mode=1, precision=1, tol=1e-10)
    g32.set_smoother(net)
    u32, i32 = g32.solve(f)
    ref, _ = osv.Solver(op, osv.Options(defl_mode=1, tol=1e-10)).solve(fh)
    e = float(np.linalg.norm(to_host(u32) - ref) / np.linalg.norm(ref))
    _say(f"[cnn train] mixed + learned at tol 1e-10: {i32['iters']} iterations, rel. difference {e:.2e}")
    assert i32["converged"] == 1 and e <= 1e-6


def test_weight_file_round_trip_and_rejects(tmp_path):
    from paper_2010_10232_amd import binding as B
    net = B.Cnn(seed=3)
    p = tmp_path / "w.hhw"
    net.save(str(p))
    back = B.Cnn(path=str(p))
    assert np.array_equal(back.get_params(), net.get_params())
    raw = bytearray(p.read_bytes())
    assert raw[:8] == b"HHCNNv1\x00" and len(raw) == 8 + 4 + 4 * net.n_floats + 8
    bad = bytearray(raw)
    bad[100] ^= 0x01
    (tmp_path / "bad.hhw").write_bytes(bytes(bad))
    with pytest.raises(B.HHError) as ei:
        B.Cnn(path=str(tmp_path / "bad.hhw"))
    assert ei.value.code == B.HH_EINVAL and "checksum" in str(ei.value)
    (tmp_path / "short.hhw").write_bytes(bytes(raw[:-3]))
    with pytest.raises(B.HHError):
        B.Cnn(path=str(tmp_path / "short.hhw"))
    with pytest.raises(B.HHError):
        B.Cnn(path=str(tmp_path / "missing.hhw"))


@pytest.mark.parametrize("name", list(CASES))
def test_fused_forward_bit_identical(name):
    """The smoother step's one-kernel forward (LDS-resident tiles of 8 x 16
    output pixels with a 4-pixel halo) against the per-layer kernels: the
    learned V-cycle gives identical bits.  The grids (101 x 101, 89 x 89,
    1 x 299) span several tiles with ragged last tiles and, in 1D, a tile taller
    than the grid."""
    from paper_2010_10232_amd import binding as B
    c, op, osol, gp, gs = build(name)
    net = B.Cnn()
    net.set_params(flat(f32_params(21, 0.2)))
    N = osol.levels[0].N
    x = np.random.default_rng(8).standard_normal(N) + 1j * np.random.default_rng(9).standard_normal(N)
    gs.set_smoother(net)
    try:
        net.set_fused(True)
        fused = to_host(gs.apply("VCYCLE", 0, to_dev(x)))
        net.set_fused(False)
        layered = to_host(gs.apply("VCYCLE", 0, to_dev(x)))
    finally:
        net.set_fused(True)
        gs.set_smoother(None)
    _say(f"[cnn case {name}] fused vs per-layer forward: max |diff| {np.max(np.abs(fused - layered)):.3e}")
    assert np.array_equal(fused, layered)
