"""The allocation-free entry point dwf_apply_normal_noalloc against
dwf_apply_normal (same kernels, so the results must agree bit for bit), on
two calls in a row, the second with a smaller lattice, in every precision;
and its size limit is reported before anything is enqueued."""
import numpy as np
import pytest

import dwfgen

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _op(dims, Ls, seed):
    import paper_2602_14454_amd as dwf
    lat = dwf.Lattice(dims)
    lat.set_gauge(dwfgen.random_su3_links(dims, 0.5, seed))
    return lat, dwf.Op(lat, Ls, 1.6, 0.03, 1.5, 0.5, 0.6)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_noalloc_matches_apply_normal_twice(prec):
    import torch
    results = []
    for dims, Ls, seed in (((8, 8, 8, 8), 12, 3), ((4, 4, 2, 6), 5, 4)):   # second call: smaller
        lat, op = _op(dims, Ls, seed)
        V = int(np.prod(dims))
        xe = _dev(dwfgen.gaussian_source_5d(dims, Ls, seed + 10)[:, : V // 2])
        ref = torch.empty_like(xe)
        op.apply_normal(ref, xe, prec=prec)
        out = torch.full_like(xe, complex(np.nan, np.nan))
        op.apply_normal_noalloc(out, xe, prec=prec)
        torch.cuda.synchronize()
        results.append((out.cpu().numpy(), ref.cpu().numpy()))
    for got, want in results:
        assert np.isfinite(got).all()
        assert np.array_equal(got, want)


def test_noalloc_rejects_lattices_beyond_its_scratch():
    import torch
    import paper_2602_14454_amd as dwf
    dims, Ls = (16, 16, 16, 16), 16   # four FP64 half fields: ~400 MB > 128 MiB
    lat, op = _op(dims, Ls, 5)
    V = int(np.prod(dims))
    xe = torch.zeros((Ls, V // 2, 4, 3), dtype=torch.complex128, device="cuda")
    out = torch.zeros_like(xe)
    with pytest.raises(dwf.DwfError) as e:
        op.apply_normal_noalloc(out, xe, prec=dwf.F64)
    assert e.value.status == -2
    # BF16 fields of the same lattice fit (4 x ~25 MB)
    op.apply_normal_noalloc(out, xe, prec=dwf.BF16)
    torch.cuda.synchronize()
    assert np.array_equal(out.cpu().numpy(), np.zeros(out.shape))
