"""Solver parity on the GPU against the FP64 oracle.

Several iterates are correct (any w with true residual <= tol), so the checks
are: the true FP64 relative residual ||y - K w|| / ||y||, recomputed by the
oracle, is <= 1e-6 in every mode; the distance to the Cholesky solution w* is
within kappa(K) x tol; and exact special cases (happy breakdown, FP64 inner CG
iterates) match the oracle closely.
"""
import numpy as np
import pytest
import torch

import oracle
from paper_1408_1237_amd import workloads

pytestmark = pytest.mark.gpu


def _api():
    from paper_1408_1237_amd import api
    return api


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.fixture(scope="module")
def small():
    p = workloads.plain_small()
    wd = oracle.direct_solve(p.x, p.sigma, p.gamma, p.y)
    K = oracle.kernel_matrix(p.x, p.sigma)
    K[np.diag_indices_from(K)] += p.gamma
    ev = np.linalg.eigvalsh(K)
    return p, wd, ev.max() / ev.min()


def test_cg64_plain_small_against_cholesky(small):
    p, wd, kappa = small
    api = _api()
    (w,), (info,) = api.krr_solve([_t(p.x)], [p.sigma], [p.gamma], [_t(p.y)], mode="cg64", max_outer=20000)
    w = w.cpu().numpy()
    assert info["status"] == 0
    rel = oracle.true_relres(p.x, p.sigma, p.gamma, p.y, w)
    assert rel <= 1e-6
    assert info["relres_true"] == pytest.approx(rel, rel=1e-3, abs=1e-12)
    assert np.linalg.norm(w - wd) / np.linalg.norm(wd) <= kappa * 1e-6
    # same algorithm and stopping rule as the oracle; with kappa ~ 1e4 the count
    # depends on rounding (summation order), so it agrees only approximately
    _, _, it_or, _, _ = oracle.cg(p.x, p.sigma, p.gamma, p.y, 20000, 1e-6)
    assert abs(info["outer_iters"] - it_or) <= max(3, 0.1 * it_or)


@pytest.mark.parametrize("inner_prec", ["fp32", "bf16", "fp64"])
@pytest.mark.parametrize("gs", ["mgs", "cgs2"])
def test_fgmres_plain_small(small, inner_prec, gs):
    p, wd, kappa = small
    api = _api()
    w, info = api.fgmres_solve(_t(p.x), p.sigma, p.gamma, _t(p.y), inner_prec=inner_prec, gs=gs,
                               inner_maxit=10)
    w = w.cpu().numpy()
    assert info["status"] == 0, info
    rel = oracle.true_relres(p.x, p.sigma, p.gamma, p.y, w)
    assert rel <= 1e-6
    assert info["relres_true"] == pytest.approx(rel, rel=1e-3, abs=1e-12)
    assert np.linalg.norm(w - wd) / np.linalg.norm(wd) <= kappa * 1e-6
    assert info["outer_iters"] >= 1 and info["inner_iters"] <= 10 * info["outer_iters"]


def test_gmres_mode_matches_oracle_gmres(small):
    p, wd, kappa = small
    api = _api()
    (w,), (info,) = api.krr_solve([_t(p.x)], [p.sigma], [p.gamma], [_t(p.y)], mode="gmres", restart_m=50,
                                  max_outer=5000)
    r = oracle.fgmres(p.x, p.sigma, p.gamma, p.y, m=50, max_outer=5000, tol=1e-6, inner="none")
    assert info["status"] == 0 and r["status"] == 0
    # FP64 on both sides with the same restart length: the step counts agree
    assert abs(info["outer_iters"] - r["outer"]) <= 2
    assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y, w.cpu().numpy()) <= 1e-6


def test_fgmres_happy_breakdown_coincident_points():
    n, gamma = 500, 0.1
    x = np.zeros((n, 3))
    api = _api()
    w, info = api.fgmres_solve(_t(x), 1.0, gamma, _t(np.ones(n)), tol=1e-12, inner="none")
    assert info["status"] == 0 and info["outer_iters"] == 1
    assert np.allclose(w.cpu().numpy(), np.ones(n) / (n + gamma), rtol=1e-13)


def test_fgmres_not_converged_returns_best_iterate(small):
    p, wd, kappa = small
    api = _api()
    from paper_1408_1237_amd import native as N
    import ctypes
    pts = N.Points(p.n, p.d, 0)
    xt, yt = _t(p.x), _t(p.y)
    w = torch.zeros_like(yt)
    o = api.make_opts(max_outer=1, tol=1e-12)
    info = N.Info()
    ws = api.workspace(N.workspace_size(N.KRR_WS_FGMRES, [(p.n, p.d)], opts=o), xt.device)
    pts = N.Points(p.n, p.d, xt.data_ptr())
    rc = N.load().fgmres_solve(ctypes.byref(pts), p.sigma, p.gamma, yt.data_ptr(), w.data_ptr(), ctypes.byref(o),
                               ctypes.byref(info), ws.data_ptr(), ws.numel(),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == N.KRR_NOT_CONVERGED and info.outer_iters == 1
    rel = oracle.true_relres(p.x, p.sigma, p.gamma, p.y, w.cpu().numpy())
    assert rel < 1.0 and info.relres_true == pytest.approx(rel, rel=1e-6)


def test_fgmres_warm_start(small):
    p, wd, kappa = small
    api = _api()
    x0 = wd * (1 + 1e-3)
    w, info = api.fgmres_solve(_t(p.x), p.sigma, p.gamma, _t(p.y), x0=_t(x0))
    assert info["status"] == 0
    assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y, w.cpu().numpy()) <= 1e-6


def test_nonfinite_input_rejected():
    api = _api()
    from paper_1408_1237_amd import native as N
    x = workloads.random_points(1, 100, 2, 1.0)
    x[17, 1] = np.nan
    with pytest.raises(N.KrrError) as e:
        api.fgmres_solve(_t(x), 0.3, 0.01, _t(np.ones(100)))
    assert e.value.code == N.KRR_ENONFINITE
    y = np.ones(100)
    y[3] = np.inf
    with pytest.raises(N.KrrError) as e:
        api.fgmres_solve(_t(workloads.random_points(1, 100, 2, 1.0)), 0.3, 0.01, _t(y))
    assert e.value.code == N.KRR_ENONFINITE


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_cg_inner_solve_matches_oracle_iterates(prec):
    # truncated CG (5 iterations, no early stop) on M = K_hat + delta I
    p = workloads.plain_small(n=1500)
    api = _api()
    dt = torch.float64 if prec == "fp64" else torch.float32
    z, info = api.cg_inner_solve(_t(p.x), p.sigma, p.delta, _t(p.y).to(dt), maxit=5, tol=0.0, prec=prec)
    zo, st, it, _, _ = oracle.cg(p.x, p.sigma, p.delta, p.y, 5, 0.0, confirm=False)
    assert info["inner_iters"] == 5 and it == 5
    err = np.linalg.norm(z.double().cpu().numpy() - zo) / np.linalg.norm(zo)
    assert err <= (1e-11 if prec == "fp64" else 2e-4)


def test_cg_inner_solve_early_stop():
    p = workloads.plain_small(n=800)
    api = _api()
    z, info = api.cg_inner_solve(_t(p.x), p.sigma, 1.0, _t(p.y).float(), maxit=200, tol=1e-4, prec="fp32")
    zo, st, it, rel, _ = oracle.cg(p.x, p.sigma, 1.0, p.y, 200, 1e-4, confirm=False)
    assert info["inner_iters"] < 200 and abs(info["inner_iters"] - it) <= 1


def test_krr_solve_several_systems_and_columns():
    api = _api()
    probs = workloads.batched(nsys=3, nmin=300, nmax=900, nrhs=2)
    Ws, infos = api.krr_solve([_t(p.x) for p in probs], [p.sigma for p in probs], [p.gamma for p in probs],
                              [torch.from_numpy(np.asfortranarray(p.y)).cuda() for p in probs], mode="fgmres")
    assert len(infos) == 6 and all(i["status"] == 0 for i in infos)
    for p, W in zip(probs, Ws):
        Wn = W.cpu().numpy()
        for r in range(2):
            assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y[:, r], Wn[:, r]) <= 1e-6


def _fcol(a):
    return torch.from_numpy(np.asfortranarray(a)).cuda()


@pytest.mark.parametrize("inner_prec", ["fp32", "bf16"])
def test_batched_mixed_dims_against_oracle(inner_prec):
    # systems of different size and dimension advance together; every column
    # must reach the true FP64 residual on its own
    api = _api()
    rng = np.random.default_rng(60)
    shapes = [(700, 2), (300, 5), (1500, 3), (257, 8)]
    xs = [np.ascontiguousarray(rng.uniform(0, 3, (n, d))) for n, d in shapes]
    ys = [np.asfortranarray(rng.standard_normal((n, 3))) for n, _ in shapes]
    sig = [0.4, 1.0, 0.3, 1.5]
    gam = [1e-2, 1e-3, 1e-2, 1e-1]
    Ws, infos = api.krr_solve([_t(x) for x in xs], sig, gam, [_fcol(y) for y in ys], mode="fgmres",
                              inner_prec=inner_prec, restart_m=60, max_outer=2000)
    assert len(infos) == 12 and all(i["status"] == 0 for i in infos), infos
    for x, y, s, g, W in zip(xs, ys, sig, gam, Ws):
        Wn = W.cpu().numpy()
        for r in range(3):
            assert oracle.true_relres(x, s, g, y[:, r], Wn[:, r]) <= 1e-6


def test_batched_matches_single_solves_and_zero_column():
    api = _api()
    probs = workloads.batched(nsys=2, nmin=600, nmax=1200, nrhs=3)
    probs[1].y[:, 1] = 0.0  # a zero right-hand side: w = 0 at once
    Ws, infos = api.krr_solve([_t(p.x) for p in probs], [p.sigma for p in probs], [p.gamma for p in probs],
                              [_fcol(p.y) for p in probs], mode="fgmres")
    assert all(i["status"] == 0 for i in infos)
    assert np.all(Ws[1].cpu().numpy()[:, 1] == 0.0)
    for p, W in zip(probs, Ws):
        for r in range(3):
            if not np.any(p.y[:, r]):
                continue
            w1, i1 = api.fgmres_solve(_t(p.x), p.sigma, p.gamma, _t(p.y[:, r]))
            a, b = W.cpu().numpy()[:, r], w1.cpu().numpy()
            # both solve to 1e-6; they agree to within the conditioning of K
            assert np.linalg.norm(a - b) / np.linalg.norm(b) <= 1e-3
            assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y[:, r], a) <= 1e-6


def test_batched_independent_of_system_order():
    # every (system, column) pair is its own FGMRES instance: permuting the
    # systems of a batch permutes the results and changes nothing else
    api = _api()
    probs = workloads.batched(nsys=3, nmin=500, nmax=1500, nrhs=2)
    order = [2, 0, 1]
    args = lambda ps: ([_t(p.x) for p in ps], [p.sigma for p in ps], [p.gamma for p in ps],
                       [_fcol(p.y) for p in ps])
    Wa, ia = api.krr_solve(*args(probs), mode="fgmres")
    Wb, ib = api.krr_solve(*args([probs[k] for k in order]), mode="fgmres")
    assert all(i["status"] == 0 for i in ia + ib)
    for pos, k in enumerate(order):
        a, b = Wa[k].cpu().numpy(), Wb[pos].cpu().numpy()
        assert np.linalg.norm(a - b) <= 1e-12 * np.linalg.norm(a)
        for r in range(2):
            assert ia[2 * k + r]["outer_iters"] == ib[2 * pos + r]["outer_iters"]


def test_batched_gmres_mode():
    api = _api()
    probs = workloads.batched(nsys=3, nmin=300, nmax=800, nrhs=2)
    Ws, infos = api.krr_solve([_t(p.x) for p in probs], [p.sigma for p in probs], [p.gamma for p in probs],
                              [_fcol(p.y) for p in probs], mode="gmres", restart_m=100, max_outer=3000)
    assert all(i["status"] == 0 for i in infos)
    for p, W in zip(probs, Ws):
        for r in range(2):
            assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y[:, r], W.cpu().numpy()[:, r]) <= 1e-6


def test_batched_graph_replays_match_eager(monkeypatch):
    # every outer step of the batched solver (inner CG, outer product,
    # Gram-Schmidt, Givens) is a recorded HIP graph per step index, replayed at
    # every cycle with eager kernels and host synchronisations between replays;
    # the arithmetic is deterministic, so the graph and eager runs agree bitwise
    # (MGS and CGS2)
    api = _api()
    probs = workloads.batched(nsys=3, nmin=400, nmax=900, nrhs=2)
    args = ([_t(p.x) for p in probs], [p.sigma for p in probs], [p.gamma for p in probs],
            [_fcol(p.y) for p in probs])
    for gs in ("mgs", "cgs2"):
        monkeypatch.setenv("KRR_NO_GRAPH", "0")
        Wg, ig = api.krr_solve(*args, mode="fgmres", gs=gs, restart_m=8)
        monkeypatch.setenv("KRR_NO_GRAPH", "1")
        We, ie = api.krr_solve(*args, mode="fgmres", gs=gs, restart_m=8)
        assert ig[0]["outer_iters"] == ie[0]["outer_iters"] and ig[0]["outer_iters"] > 8  # several cycles
        for a, b in zip(Wg, We):
            assert torch.equal(a, b)


def _bargs(probs):
    return ([_t(p.x) for p in probs], [p.sigma for p in probs], [p.gamma for p in probs],
            [_fcol(p.y) for p in probs])


def test_batched_cgs2_and_per_column_counts():
    # classical Gram-Schmidt twice in the batched solver; every column keeps its
    # own outer count (columns stop on their own), its FP64 product count is its
    # steps plus one true residual per cycle, and the batch ran as many steps as
    # its slowest column (at most cg_check more: the host checks every cg_check)
    api = _api()
    probs = workloads.batched(nsys=3, nmin=400, nmax=1400, nrhs=3)
    Ws, infos = api.krr_solve(*_bargs(probs), mode="fgmres", gs="cgs2", restart_m=40, cg_check=4)
    assert all(i["status"] == 0 for i in infos), infos
    for p, W in zip(probs, Ws):
        for r in range(3):
            assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y[:, r], W.cpu().numpy()[:, r]) <= 1e-6
    outer = [i["outer_iters"] for i in infos]
    assert len(set(outer)) > 1
    for i in infos:
        assert i["mvp64"] == i["outer_iters"] + i["cycles"]
        assert i["mvp32"] == i["inner_iters"] and 0 < i["inner_iters"] <= 10 * i["outer_iters"]
        assert i["batch_steps"] >= max(outer) and i["batch_tiles"] in (16, 32, 64, 128)
    # MGS on the same batch reaches the same tolerance
    Wm, im = api.krr_solve(*_bargs(probs), mode="fgmres", gs="mgs", restart_m=40)
    assert all(i["status"] == 0 for i in im)


def test_batched_fp64_inner_products_are_honoured():
    # FP64 inner products are not batched: the pairs are solved one at a time
    # with FP64 inner CG (no FP32 / BF16 products), each to the tolerance
    api = _api()
    probs = workloads.batched(nsys=2, nmin=300, nmax=700, nrhs=2)
    Ws, infos = api.krr_solve(*_bargs(probs), mode="fgmres", inner_prec="fp64")
    for p, W, k in zip(probs, Ws, range(2)):
        for r in range(2):
            i = infos[2 * k + r]
            assert i["status"] == 0 and i["mvp32"] == 0 and i["mvp16"] == 0 and i["batch_steps"] == 0
            assert i["mvp64"] > i["outer_iters"]  # inner and outer products both FP64
            assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y[:, r], W.cpu().numpy()[:, r]) <= 1e-6


@pytest.mark.parametrize("mode", ["fgmres", "cg64"])
def test_batched_nonfinite_column_is_retired_alone(mode):
    # a right-hand side with a NaN: that column is not solved (zero, status
    # KRR_ENONFINITE), every other column is, and the call reports KRR_ENONFINITE
    from paper_1408_1237_amd import native
    api = _api()
    probs = workloads.batched(nsys=2, nmin=400, nmax=900, nrhs=3)
    probs[0].y[5, 1] = np.nan
    Ws, infos, rc = api.krr_solve(*_bargs(probs), mode=mode, return_status=True, max_outer=5000)
    assert rc == native.KRR_ENONFINITE
    assert infos[1]["status"] == native.KRR_ENONFINITE
    assert np.all(Ws[0].cpu().numpy()[:, 1] == 0.0)
    for k, p in enumerate(probs):
        for r in range(3):
            if (k, r) == (0, 1):
                continue
            assert infos[3 * k + r]["status"] == 0
            assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y[:, r], Ws[k].cpu().numpy()[:, r]) <= 1e-6


def test_batched_cg64_matches_single_cg64():
    # plain FP64 CG over every (system, column) pair at once: each column to the
    # true residual 1e-6, with about the iterations of its own single CG solve
    api = _api()
    probs = workloads.batched(nsys=3, nmin=300, nmax=1200, nrhs=2)
    Ws, infos = api.krr_solve(*_bargs(probs), mode="cg64", max_outer=20000, cg_check=8)
    assert all(i["status"] == 0 and i["batch_steps"] > 0 for i in infos), infos
    for k, (p, W) in enumerate(zip(probs, Ws)):
        for r in range(2):
            i = infos[2 * k + r]
            y = np.ascontiguousarray(p.y[:, r])
            assert oracle.true_relres(p.x, p.sigma, p.gamma, y, W.cpu().numpy()[:, r]) <= 1e-6
            (w1,), (i1,) = api.krr_solve([_t(p.x)], [p.sigma], [p.gamma], [_t(y)], mode="cg64", max_outer=20000)
            assert abs(i["outer_iters"] - i1["outer_iters"]) <= max(3, 0.1 * i1["outer_iters"])
            assert i["mvp64"] >= i["outer_iters"] + 1


@pytest.mark.parametrize("tps", ["16", "128"])
def test_batched_work_item_tile_does_not_change_the_solution(monkeypatch, tps):
    # KRR_BATCH_TPS fixes the column tiles per work item (else autotuned); the
    # partial sums change with it only at rounding level
    api = _api()
    probs = workloads.batched(nsys=2, nmin=4000, nmax=9000, nrhs=2)
    monkeypatch.delenv("KRR_BATCH_TPS", raising=False)
    Wa, ia = api.krr_solve(*_bargs(probs), mode="fgmres")
    monkeypatch.setenv("KRR_BATCH_TPS", tps)
    Wb, ib = api.krr_solve(*_bargs(probs), mode="fgmres")
    assert all(i["status"] == 0 for i in ia + ib)
    assert all(i["batch_tiles"] == int(tps) for i in ib)
    for p, a, b in zip(probs, Wa, Wb):
        for r in range(2):
            assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y[:, r], b.cpu().numpy()[:, r]) <= 1e-6
        assert torch.linalg.norm(a - b) <= 1e-3 * torch.linalg.norm(a)


def test_cg64_workspace_holds_the_coefficient_history():
    # the plain CG keeps two coefficients per iteration for the condition
    # estimate: at small n with a large iteration cap that history is larger
    # than the flexible solvers' basis, and the solve workspace covers it
    api = _api()
    p = workloads.plain_small(n=300)
    (w,), (info,) = api.krr_solve([_t(p.x)], [p.sigma], [p.gamma], [_t(p.y)], mode="cg64", max_outer=60000)
    assert info["status"] == 0
    assert oracle.true_relres(p.x, p.sigma, p.gamma, p.y, w.cpu().numpy()) <= 1e-6
