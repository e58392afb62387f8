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
    assert o.precision == 0 and o.time_kernels == 0 and o.autotune == 1


@pytest.mark.parametrize("kw", [dict(dim=3, p=2, n_el=8, k=1.0), dict(dim=2, p=0, n_el=8, k=1.0),
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


@pytest.mark.parametrize("dim,p,n", [(1, 2, 80), (2, 3, 160), (2, 4, 7), (2, 1, 5)])
def test_problem_sizes(dim, p, n):
    pr = B.Problem(dim, p, n, k=10.0)
    if dim == 1:
        assert pr.n == (n + p - 2, 1)
    else:
        assert pr.n == (n + p - 2, n + p - 2)


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
