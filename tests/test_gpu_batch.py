"""Batched solves on the GPU (dwf_solve_batch): every right-hand side of
every operator in the batch must solve its own 5D system.  The FP64 oracle
recomputes the true residual |b5 - D x5| / |b5| of each GPU solution with its
own operator (full spin matrices, block table of the Neff form); it must be
within the requested tolerance.  Schedules that only change how the work is
distributed (graph replay, right-hand sides per block, block order) must give
bit-identical solutions."""
import numpy as np
import pytest

import dwfgen
import oracle

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _point_sources(op, dims, Ls, spins=range(4), colours=range(3)):
    """b5 of the spin-colour point sources at the origin, built on the GPU."""
    import torch
    V = int(np.prod(dims))
    srcs = [(s, c) for s in spins for c in colours]
    b5 = torch.empty((len(srcs), Ls, V, 4, 3), dtype=torch.complex128, device="cuda")
    for k, (s, c) in enumerate(srcs):
        op.source_4d(b5[k], _dev(dwfgen.point_source_4d(dims, s, c)))
    return b5


def _oracle_res(case, U, x5, b5):
    dims, Ls, M0, m, b, c, al = case
    p = oracle.Params(dims=dims, Ls=Ls, M0=M0, m=m, b=b, c=c, alpha=al)
    return oracle.true_residual(p, U, x5, b5)


def _ops(cases, seed0=100):
    import paper_2602_14454_amd as dwf
    out = []
    for k, case in enumerate(cases):
        dims, Ls, M0, m, b, c, al = case
        U = dwfgen.make_links(dims, 0.5, seed0 + k, rho=0.1, nsmear=1)
        lat = dwf.Lattice(dims)
        lat.set_gauge(U)
        out.append((case, U, lat, dwf.Op(lat, Ls, M0, m, b, c, al)))
    return out


@pytest.fixture(autouse=True)
def _memory_tune_cache(monkeypatch):
    import paper_2602_14454_amd as dwf
    monkeypatch.setenv("DWF_TUNE_CACHE", "off")
    dwf.tune_cache_reload()
    yield
    dwf.tune_cache_reload()


@pytest.mark.parametrize("prec", [1, 2])
def test_twelve_point_sources(prec):
    """12 spin-colour point sources of one operator in one batched solve."""
    import torch
    import paper_2602_14454_amd as dwf
    case = ((6, 4, 4, 8), 8, 1.6, 0.02, 1.0, 0.0, 0.5)
    (_, U, lat, op), = _ops([case])
    b5 = _point_sources(op, case[0], case[1])
    x5 = torch.zeros_like(b5)
    prm = dwf.default_params(algo=dwf.ALGO_DC, inner_prec=prec, check_every=4, tol=1e-10)
    st, infos = dwf.solve_batch([op], [x5], [b5], [12], prm)
    assert st == 0 and len(infos) == 12
    xh, bh = x5.cpu().numpy(), b5.cpu().numpy()
    for k, f in enumerate(infos):
        assert f.converged and f.true_res5 <= 1e-10 and f.iters > 0
        assert _oracle_res(case, U, xh[k], bh[k]) <= 1.2e-10
    # the same slot solved alone (single-solve path, FP64 CGNR) gives the same x5
    xs = torch.zeros_like(b5[5])
    op.solve(xs, b5[5], dwf.default_params(tol=1e-12, check_every=4))
    rel = (torch.linalg.vector_norm(x5[5] - xs) / torch.linalg.vector_norm(xs)).item()
    assert rel < 1e-7
    # and a batched slot takes no more inner iterations than the single-solve
    # defect correction with the same parameters (both test convergence at
    # multiples of the check period; rounding may move a test by one period
    # per outer step)
    xs.zero_()
    st1, f1 = op.solve(xs, b5[5], prm)
    assert st1 == 0
    slack = 4 * max(f1.outer_iters, infos[5].outer_iters)
    assert infos[5].iters <= f1.iters + slack, (infos[5].iters, f1.iters)


UNEVEN = [
    ((4, 4, 4, 4), 8, 1.6, 0.05, 1.0, 0.0, 1.0),     # KK = 2
    ((6, 6, 2, 2), 12, 1.8, 0.03, 1.5, 0.5, 0.6),    # KK = 3, Vh = 72 (ragged tile)
    ((4, 4, 4, 8), 16, 1.6, 0.01, 1.0, 0.0, 0.5),    # KK = 4
    ((2, 2, 4, 4), 4, 1.6, 0.02, 1.0, 1.0, 0.7),     # KK = 1, Mobius (b, c) = (1, 1)
    ((4, 4, 2, 6), 7, 1.7, 0.005, 1.2, 0.3, 0.8),    # KK = 2, Ls odd
]


@pytest.mark.parametrize("algo,prec", [(1, 1), (1, 2), (0, 0)])
def test_uneven_batch(algo, prec):
    """Lattices of different size, Ls, mass, (b, c) and alpha in one batch,
    one and two right-hand sides."""
    import torch
    import paper_2602_14454_amd as dwf
    objs = _ops(UNEVEN)
    nrhs = [1, 2, 1, 2, 1]
    xs, bs = [], []
    for (case, U, lat, op), k in zip(objs, nrhs):
        dims, Ls = case[0], case[1]
        b = np.stack([dwfgen.gaussian_source_5d(dims, Ls, 50 + 7 * j + Ls) for j in range(k)])
        bs.append(_dev(b))
        xs.append(torch.zeros_like(bs[-1]))
    prm = dwf.default_params(algo=algo, inner_prec=prec, check_every=4, tol=1e-10)
    st, infos = dwf.solve_batch([o[3] for o in objs], xs, bs, nrhs, prm)
    assert st == 0 and len(infos) == sum(nrhs)
    slot = 0
    for (case, U, lat, op), x, b, k in zip(objs, xs, bs, nrhs):
        xh, bh = x.cpu().numpy(), b.cpu().numpy()
        for j in range(k):
            f = infos[slot]
            assert f.converged and f.true_res5 <= 1e-10
            assert _oracle_res(case, U, xh[j], bh[j]) <= 1.2e-10
            slot += 1
    # each slot stops on its own test
    assert len({f.iters for f in infos}) > 1


def test_schedules_are_bit_identical():
    """Graph replay vs eager launches and every tile schedule of the
    work-list hop produce the same bits, for check periods 4, 20 and 1 (the
    direction ring is 4, 16 or 1 long; a period of 20 wraps it once inside
    the period).  Slots test convergence at multiples of the check period,
    as the single solve does, so the period itself may change the result."""
    import torch
    import paper_2602_14454_amd as dwf
    objs = _ops(UNEVEN[:3], seed0=300)
    nrhs = [3, 1, 2]
    bs = []
    for (case, U, lat, op), k in zip(objs, nrhs):
        dims, Ls = case[0], case[1]
        bs.append(_dev(np.stack([dwfgen.gaussian_source_5d(dims, Ls, 90 + j) for j in range(k)])))
    ops = [o[3] for o in objs]
    key = "gfx950|p1|" + "|".join(f"{o[0][0][0]}x{o[0][0][1]}x{o[0][0][2]}x{o[0][0][3]}s{o[0][1]}r{k}"
                                  for o, k in zip(objs, nrhs))
    ref = {}
    for nrb, order, graph, every in [(1, 0, 1, 4), (1, 0, 0, 4), (2, 1, 1, 4), (3, 0, 1, 4), (3, 1, 0, 4),
                                     (1, 0, 1, 20), (2, 1, 0, 20), (1, 0, 1, 1), (3, 0, 0, 1)]:
        dwf.tune_cache_put(key, nrb, order, 1.0)
        xs = [torch.zeros_like(b) for b in bs]
        prm = dwf.default_params(algo=dwf.ALGO_DC, inner_prec=dwf.F32, check_every=every, autotune=0,
                                 use_graph=graph)
        st, infos = dwf.solve_batch(ops, xs, bs, nrhs, prm)
        assert st == 0
        res = ([x.cpu().numpy() for x in xs], [f.iters for f in infos])
        if every not in ref:
            ref[every] = res
        else:
            assert res[1] == ref[every][1]
            for a, b in zip(res[0], ref[every][0]):
                assert np.array_equal(a, b)
    for every, (_, iters) in ref.items():
        # each inner solve ends at a multiple of the check period
        assert all(k % every == 0 for k in iters), (every, iters)


def test_zero_source_slot_and_autotune():
    """A zero right-hand side converges at once with x = 0 (no NaN); the tuner
    returns a valid schedule and stores it."""
    import torch
    import paper_2602_14454_amd as dwf
    (case, U, lat, op), = _ops([UNEVEN[0]], seed0=500)
    dims, Ls = case[0], case[1]
    b = np.stack([dwfgen.gaussian_source_5d(dims, Ls, 3), np.zeros((Ls, int(np.prod(dims)), 4, 3), np.complex128)])
    bd = _dev(b)
    x = torch.zeros_like(bd)
    st, infos = dwf.solve_batch([op], [x], [bd], [2], dwf.default_params(algo=dwf.ALGO_DC, check_every=4))
    assert st == 0
    assert infos[1].converged and infos[1].iters == 0 and torch.count_nonzero(x[1]).item() == 0
    assert infos[0].true_res5 <= 1e-10
    nrb, order, ms = dwf.autotune_batch([op], [2], dwf.F32)
    assert nrb in (1, 2) and order in (0, 1) and ms > 0
    key = f"gfx950|p1|{dims[0]}x{dims[1]}x{dims[2]}x{dims[3]}s{Ls}r2"
    assert dwf.tune_cache_get(key)[:2] == (nrb, order)


def test_batch_rejects_bad_arguments():
    import torch
    import paper_2602_14454_amd as dwf
    (case, U, lat, op), = _ops([UNEVEN[0]], seed0=600)
    x = torch.zeros((1, case[1], 256, 4, 3), dtype=torch.complex128, device="cuda")
    with pytest.raises(dwf.DwfError):
        dwf.solve_batch([op], [x], [x], [0])
    with pytest.raises(dwf.DwfError):
        dwf.solve_batch([op], [x], [x], [1], dwf.default_params(algo=dwf.ALGO_MIXED))


def test_batch_nan_source_reports_enan():
    """A NaN in one right-hand side of a batch stops the batch with DWF_ENAN
    (the other operator of the batch is still iterating when it is seen),
    and a later batch on the same operators solves normally."""
    import torch
    import paper_2602_14454_amd as dwf
    objs = _ops(UNEVEN[:2], seed0=700)
    bs, xs = [], []
    for k, (case, U, lat, op) in enumerate(objs):
        dims, Ls = case[0], case[1]
        b = np.stack([dwfgen.gaussian_source_5d(dims, Ls, 40 + k)])
        if k == 1:
            b[0, 2, 1, 0, 0] = np.nan
        bs.append(_dev(b))
        xs.append(torch.zeros_like(bs[-1]))
    ops = [o[3] for o in objs]
    prm = dwf.default_params(algo=dwf.ALGO_DC, inner_prec=dwf.F32, check_every=4, tol=1e-10)
    with pytest.raises(dwf.DwfError) as e:
        dwf.solve_batch(ops, xs, bs, [1, 1], prm)
    assert e.value.status == -6
    bs[1] = _dev(np.stack([dwfgen.gaussian_source_5d(objs[1][0][0], objs[1][0][1], 41)]))
    xs = [torch.zeros_like(b) for b in bs]
    st, infos = dwf.solve_batch(ops, xs, bs, [1, 1], prm)
    assert st == 0 and all(f.converged for f in infos)


def test_batch_iteration_budget():
    """With an iteration budget far below what the solves need, every slot
    stops within one check period of the budget and the batch reports
    DWF_NOT_CONVERGED (1) with finite, improved iterates."""
    import torch
    import paper_2602_14454_amd as dwf
    objs = _ops(UNEVEN[:3], seed0=800)
    bs = []
    for k, (case, U, lat, op) in enumerate(objs):
        dims, Ls = case[0], case[1]
        bs.append(_dev(np.stack([dwfgen.gaussian_source_5d(dims, Ls, 60 + k)])))
    xs = [torch.zeros_like(b) for b in bs]
    prm = dwf.default_params(algo=dwf.ALGO_DC, inner_prec=dwf.F32, check_every=4, tol=1e-10, maxiter=12)
    st, infos = dwf.solve_batch([o[3] for o in objs], xs, bs, [1, 1, 1], prm)
    assert st == 1
    for f, x in zip(infos, xs):
        assert f.converged == 0 and 0 < f.iters <= 12 + 4
        assert 0 < f.true_res5 < 1.0 and torch.isfinite(x).all()
