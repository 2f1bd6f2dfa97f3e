"""GPU: the no-allocation apply (msc_op_apply_noalloc) against msc_op_apply.

Two calls in a row on one device, the second with a smaller operator, for both kinds
and both precisions: the outputs equal those of the allocating entry point bit for bit
(same kernels, same lane count, temporaries in the library's fixed device array instead
of the operator's workspace).  An operator beyond the array's limit is rejected.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _systems():
    big = W.staggered_problem((8, 8, 8, 8), 0.1, 71, 72, (1e-3, 1.0, 2))
    small = W.staggered_problem((4, 4, 4, 4), 0.1, 73, 74, (1e-3, 1.0, 2))
    rp, col, vals = W.laplacian7_csr((12, 10, 9), 75)
    lap_big = dict(kind="herm", n=12 * 10 * 9, rowptr=rp, col=col, vals=vals)
    rp, col, vals = W.laplacian7_csr((5, 4, 3), 76)
    lap_small = dict(kind="herm", n=60, rowptr=rp, col=col, vals=vals)
    return [(big, small), (lap_big, lap_small)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_noalloc_apply_matches_apply_twice_shrinking(cuda, prec):
    import torch
    from paper_1102_2143_amd import Operator
    for pair in _systems():
        for call, p in enumerate(pair):
            print(f"[gpu] apply_noalloc {prec} kind={p['kind']} n={p['n']} call={call}",
                  flush=True)
            op = Operator(p["rowptr"], p["col"], p["vals"], p["n"], kind=p["kind"],
                          device=cuda)
            v = torch.from_numpy(W.gaussian_rhs(p["n"], 100 + call)).to(cuda)
            ref = op.apply(v, shift=0.37, prec=prec)
            out = torch.full((p["n"],), complex("nan"), dtype=torch.complex128, device=cuda)
            op.apply_noalloc(v, out, shift=0.37, prec=prec)
            torch.cuda.synchronize()
            assert torch.equal(out, ref), (prec, p["kind"], p["n"])
            op.close()


def test_noalloc_apply_rejects_operators_beyond_its_scratch(cuda):
    import torch
    from paper_1102_2143_amd import MscError, Operator
    # FP64 with A = M^H M needs two complex128 temporaries: 2^21 + 1 rows exceed 64 MiB
    n = (1 << 21) + 1
    rowptr = np.arange(n + 1, dtype=np.int64)
    col = np.arange(n, dtype=np.int32)
    vals = np.full(n, 2.0 + 0.0j)
    print(f"[gpu] apply_noalloc rejection n={n}", flush=True)
    op = Operator(rowptr, col, vals, n, kind="mhm", device=cuda)
    v = torch.ones(n, dtype=torch.complex128, device=cuda)
    out = torch.empty_like(v)
    with pytest.raises(MscError):
        op.apply_noalloc(v, out, prec="fp64")
    # the complex64 temporaries of the same operator fit: (A + 1) v = 5 v exactly
    op.apply_noalloc(v, out, shift=1.0, prec="mixed")
    torch.cuda.synchronize()
    assert torch.equal(out, torch.full_like(v, 5.0))
    op.close()
