"""C ABI checks that need no GPU: the library loads, exports every declared
entry point, and its host-side problem set-up agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2010_10232_amd import binding as B
from oracle import helmholtz as hz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "hh.h")).read()
    return sorted(set(re.findall(r"^\s*(?:hh_status|void|const char\*)\s+(hh_\w+)\s*\(", src, re.M)))


def test_library_exports_every_declared_symbol():
    lib = B.load()
    names = declared_functions()
    assert len(names) >= 12
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(B.EXPORTED)


def test_default_opts():
    o = B.default_opts()
    assert (o.beta[0], o.beta[1]) == (1.0, 0.5)
    assert o.omega == 0.8 and o.restart == 50 and o.tol == 1e-7 and o.maxit == 1000
    assert list(o.defl_inner_its) == [8, 4, 2, 1, 1, 1, 1, 1]
    assert o.defl_direct_max == 16384 and o.coarse_damping == 1 and o.defl_mode == 2
    assert o.precision == 0 and o.time_kernels == 0 and o.autotune == 1 and o.ortho == 0


@pytest.mark.parametrize("kw", [dict(dim=4, p=2, n_el=8, k=1.0), dict(dim=2, p=0, n_el=8, k=1.0),
                                dict(dim=3, p=2, n_el=(8, 8, 1), k=1.0),
                                dict(dim=3, p=2, n_el=4, k_elem=np.ones((4, 4, 4))),
                                dict(dim=2, p=6, n_el=8, k=1.0), dict(dim=2, p=2, n_el=1, k=1.0),
                                dict(dim=2, p=2, n_el=8, k=-1.0), dict(dim=2, p=2, n_el=8, k=float("nan"))])
def test_assemble_rejects_invalid(kw):
    with pytest.raises(B.HHError) as e:
        B.Problem(**kw)
    assert e.value.code == B.HH_EINVAL


def test_assemble_rejects_bad_k_field():
    k = np.full((4, 4), 3.0)
    k[1, 2] = 0.0
    with pytest.raises(B.HHError):
        B.Problem(2, 2, 4, k_elem=k)


@pytest.mark.parametrize("dim,p,n", [(1, 2, 80), (2, 3, 160), (2, 4, 7), (2, 1, 5), (3, 2, 9), (3, 5, 4)])
def test_problem_sizes(dim, p, n):
    pr = B.Problem(dim, p, n, k=10.0)
    if dim == 1:
        assert pr.n == (n + p - 2, 1)
    elif dim == 2:
        assert pr.n == (n + p - 2, n + p - 2)
    else:
        assert pr.n == (n + p - 2,) * 3 and pr.N == (n + p - 2) ** 3
        with pytest.raises(B.HHError):      # two sizes cannot describe the cube
            B._check(B.load().hh_problem_size(pr._h, (ctypes.c_int * 2)()))


def test_problem_sizes_3d_anisotropic():
    pr = B.Problem(3, 3, (5, 7, 6), k=4.0)
    assert pr.n == (6, 8, 7) and pr.N == 6 * 8 * 7
    assert pr.spans((0.23, 0.61, 0.82)) == [1, 4, 4]


@pytest.mark.parametrize("x0", [(0.5, 0.95), (0.0, 1.0), (1.0, 0.5), (0.3, 0.7), (0.999999, 1e-9),
                                (3 / 7, 0.625)])
@pytest.mark.parametrize("n_el", [480, 7, 160])
def test_point_spans_bit_exact(x0, n_el):
    pr = B.Problem(2, 3, n_el, k=10.0)
    op = hz.Problem(2, 3, n_el, 10.0)
    assert pr.spans(x0) == hz.source_spans(op, x0)


def test_point_spans_reject_outside():
    pr = B.Problem(2, 3, 16, k=10.0)
    for x0 in [(-0.1, 0.5), (0.5, 1.0000001)]:
        with pytest.raises(B.HHError):
            pr.spans(x0)


_CSR_CASES = [
    dict(dim=1, p=2, n_el=20, k=7.0),
    dict(dim=1, p=5, n_el=13, rand=True),
    dict(dim=2, p=1, n_el=6, k=3.0),
    dict(dim=2, p=3, n_el=12, k=9.0),
    dict(dim=2, p=2, n_el=9, rand=True),
    dict(dim=2, p=4, n_el=11, rand=True),
    dict(dim=1, p=3, n_el=17, k=5.0, lengths=(2.5,)),
    dict(dim=2, p=2, n_el=(9, 6), k=3.0, lengths=(2.0, 0.75)),
    dict(dim=2, p=3, n_el=(8, 10), rand=True, lengths=(0.5, 1.5)),
    dict(dim=3, p=2, n_el=(3, 4, 2), k=4.0, lengths=(1.5, 0.5, 2.0)),
    dict(dim=3, p=1, n_el=(4, 3, 5), k=2.0),
    dict(dim=3, p=2, n_el=(3, 4, 2), k=5.0),
    dict(dim=3, p=3, n_el=(4, 3, 3), k=3.0),
]


@pytest.mark.parametrize("c", _CSR_CASES, ids=lambda c: f"d{c['dim']}p{c['p']}n{'x'.join(map(str, np.atleast_1d(c['n_el'])))}{'rand' if c.get('rand') else ''}")
def test_export_csr_matches_oracle(c):
    """Finest-level K, M_k and A exported by the library (host) against the
    oracle's scipy assembly: identical sparsity (row pointers and column
    indices bit for bit) against the oracle's nonzero pattern (scipy's kron
    stores explicit zeros of its block format, removed first), values within
    1e-13 of the largest entry."""
    ke = None
    if c.get("rand"):
        rng = np.random.default_rng(5)
        shape = tuple(np.atleast_1d(c["n_el"])[::-1]) if not np.isscalar(c["n_el"]) else (c["n_el"],) * c["dim"]
        ke = 4.0 * (1.0 + 0.5 * rng.random(shape))
    k = c.get("k", 1.0)
    gp = B.Problem(c["dim"], c["p"], c["n_el"], k=k, k_elem=ke, lengths=c.get("lengths"))
    op = hz.Problem(c["dim"], c["p"], c["n_el"], k, k_elem=ke, lengths=c.get("lengths"))
    K, Mk = hz.fine_operators(op)
    for which, ref in ((0, K), (1, Mk), (2, (K - Mk))):
        ref = ref.tocsr()
        ref.eliminate_zeros()
        ref.sort_indices()
        indptr, indices, data = gp.export_csr(which)
        assert np.array_equal(indptr, ref.indptr.astype(np.int64)), which
        assert np.array_equal(indices, ref.indices.astype(np.int32)), which
        scale = np.max(np.abs(ref.data))
        assert np.max(np.abs(data - ref.data)) <= 1e-13 * scale, which


def test_export_csr_capacity_checked():
    gp = B.Problem(2, 2, 6, k=2.0)
    lib = B.load()
    nnz = ctypes.c_longlong()
    assert lib.hh_export_csr(gp._h, 0, ctypes.byref(nnz), None, None, None, 0) == 0
    ptr = np.empty(gp.N + 1, dtype=np.int64)
    idx = np.empty(nnz.value, dtype=np.int32)
    val = np.empty(nnz.value, dtype=np.float64)
    assert lib.hh_export_csr(gp._h, 0, ctypes.byref(nnz), ptr.ctypes.data, idx.ctypes.data, val.ctypes.data,
                             nnz.value - 1) < 0
    assert lib.hh_export_csr(gp._h, 3, ctypes.byref(nnz), None, None, None, 0) < 0



@pytest.mark.parametrize("x0", [(0.0, 0.0), (2.0, 0.75), (1.3, 0.2), (0.999, 0.5), (1e-9, 0.7499999)])
def test_point_spans_on_a_rectangle_bit_exact(x0):
    pr = B.Problem(2, 3, (10, 7), k=4.0, lengths=(2.0, 0.75))
    op = hz.Problem(2, 3, (10, 7), 4.0, lengths=(2.0, 0.75))
    assert pr.spans(x0) == hz.source_spans(op, x0)


def test_lengths_checked():
    with pytest.raises(B.HHError):
        B.Problem(2, 2, 8, k=1.0, lengths=(1.0, -2.0))
    with pytest.raises(B.HHError):
        B.Problem(2, 2, 8, k=1.0, lengths=(float("nan"), 1.0))
    pr = B.Problem(2, 2, 8, k=1.0, lengths=(2.0, 0.5))
    with pytest.raises(B.HHError):
        pr.spans((1.0, 0.6))   # outside [0, 2] x [0, 0.5]
