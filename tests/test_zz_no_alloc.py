"""The allocation-free point-source entry point against the regular one.

hh_rhs_point_source_noalloc stages the two 1D basis factors in a fixed device
array instead of a per-call allocation; its load must equal hh_rhs_point_source's
bit for bit (both evaluate amp * fy[i2] * fx[i1] in the same order), also on a
second call with a smaller problem, where the array still holds the first
call's longer staging.
"""
import numpy as np
import pytest

from paper_2010_10232_amd import binding as B

pytestmark = pytest.mark.gpu


def _pair(prob, x0, amp):
    import torch
    ref = prob.point_source(x0, amp=amp)
    out = torch.full_like(ref, complex(np.nan, np.nan))
    prob.point_source_noalloc(x0, out, amp=amp)
    torch.cuda.synchronize()
    return ref.cpu().numpy(), out.cpu().numpy()


def test_noalloc_point_source_matches_regular_twice():
    import torch
    torch.cuda.set_device(0)
    # first call: a 2D workload grid (962 x 962 unknowns); second: a smaller, ragged 1D+2D pair
    cases = [((2, 4, 960, 300.0), (0.5, 0.5), 1.0),
             ((2, 3, (37, 23), 40.0), (0.31, 0.77), -2.5),
             ((1, 2, 80, 50.0), (0.5,), 1.0)]
    for (dim, p, n_el, k), x0, amp in cases:
        print(f"[no_alloc] dim={dim} p={p} n_el={n_el} x0={x0}", flush=True)
        prob = B.Problem(dim, p, n_el, k=k)
        ref, out = _pair(prob, x0, amp)
        assert out.shape == ref.shape
        assert np.array_equal(out.view(np.uint64), ref.view(np.uint64))
        nz = np.count_nonzero(ref)
        assert 0 < nz <= (p + 1) ** dim
        prob.close()


def test_noalloc_point_source_rejects_oversize():
    import torch
    torch.cuda.set_device(0)
    prob = B.Problem(1, 2, 70000, k=10.0)   # n1 + n2 = 70001 > 65536
    dummy = torch.zeros(4, dtype=torch.complex128, device="cuda")
    with pytest.raises(B.HHError) as ei:
        prob.point_source_noalloc((0.5,), dummy)
    assert ei.value.code == B.HH_EINVAL and "capacity" in str(ei.value)
    assert torch.count_nonzero(dummy).item() == 0
    prob.close()
