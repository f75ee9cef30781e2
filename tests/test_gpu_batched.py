"""GPU parity of the batched sweeps (inner product + junction of
the contraction over the last two positions, per pair) against the FP64
oracle, through the C ABI: a small uneven batch and the whole 4096-pair
batch, every pair checked (FP32 and BF16 inputs, every schedule), the
per-pair launch loop, and run-to-run determinism."""
import math

import numpy as np
import pytest

from oracle import tt_oracle as O
from ttgen import configs as C

from helpers import TOL, rel_err, scalar_err, to_gpu, to_np, tt_norm

pytestmark = pytest.mark.gpu


def _oracle_pair(x, y):
    N = len(x)
    z = O.inner_lr(x, y)
    K = O.sweep_rl(x, y, downto=N - 2)[N - 2]
    return z, K


def _check_pairs(plan, inner, junc, cores64, idx, tol):
    worst = 0.0
    for p in idx:
        x, y = cores64[p]
        z, K = _oracle_pair(x, y)
        e = scalar_err(float(inner[p]), z, tt_norm(x), tt_norm(y))
        ek = rel_err(to_np(plan.junction(junc, p)), K)
        worst = max(worst, e, ek)
        assert e <= tol, (p, e)
        assert ek <= tol, (p, ek)
    return worst


# Arithmetic-only bound for BF16 cores (against the oracle on the rounded
# values): FP32 steps round at 2^-24 per operation; the BF16-MFMA schedule
# carries the interface and each per-index product as a BF16 hi / lo pair
# (16 significant bits), so each of a sweep's <= 12 steps adds about 2^-17
# relative, and 1e-4 leaves a wide margin over the ~1e-5 worst case.
ARITH_BF16 = {"lds1b": 1e-4}
ARITH_BF16_DEFAULT = 1e-5


@pytest.fixture(params=["lds1", "lds1b", "lds", "levels", "persistent"])
def batch_mode(request, monkeypatch):
    """Every batched schedule (the autotuner picks one by timing)."""
    monkeypatch.setenv("TTC_BATCH_MODE", request.param)
    return request.param


def _skip_f32_only_bf16(batch_mode, dtype):
    if batch_mode == "lds1b" and dtype != "bf16":
        pytest.skip("the BF16-MFMA schedule takes BF16 cores only")


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batch_small_uneven(ttc, dtype, batch_mode):
    _skip_f32_only_bf16(batch_mode, dtype)
    shapes = C.batch_pair_shapes(C.SEED_BATCH, 40)
    # plus degenerate shapes: order 3 with rank-1 bonds, order 12 small ranks
    shapes.append((C.TTShape([4, 4, 4], [1, 1, 1, 1]), C.TTShape([4, 4, 4], [1, 1, 1, 1])))
    shapes.append((C.TTShape([5] * 12, [1] + [3] * 11 + [1]), C.TTShape([5] * 12, [1] + [2] * 11 + [1])))
    cores64, seen, gpu = [], [], []
    for p, (sx, sy) in enumerate(shapes):
        x = C.gen_tt_np(C.SEED_BATCH, 1 + 2 * p, sx)
        y = C.gen_tt_np(C.SEED_BATCH, 2 + 2 * p, sy)
        xg, xs = to_gpu(x, dtype)
        yg, ys = to_gpu(y, dtype)
        cores64.append((x, y) if dtype == "bf16" else (xs, ys))
        seen.append((xs, ys))
        gpu.append((xg, yg))
    plan = ttc.BatchPlan(gpu)
    if batch_mode in ("lds1", "lds1b", "lds", "levels", "persistent"):
        assert plan.config["mode"] == batch_mode
    inner, junc = plan.run()
    inner = to_np(inner)
    _check_pairs(plan, inner, junc, cores64, range(len(shapes)), TOL[dtype])
    if dtype == "bf16":
        # arithmetic only: against the oracle on the values the GPU holds
        _check_pairs(plan, inner, junc, seen, range(len(shapes)), ARITH_BF16.get(batch_mode, ARITH_BF16_DEFAULT))
    # the per-pair launch loop meets the same bar
    inner2, junc2 = plan.run(plain=True)
    _check_pairs(plan, to_np(inner2), junc2, cores64, range(len(shapes)), TOL[dtype])
    # determinism of the batched launch (graph replay)
    inner3, junc3 = plan.outputs()
    plan.run(inner3, junc3)
    plan.run(inner3, junc3)
    assert np.array_equal(to_np(inner3), inner)


def test_batch_integer_cores_exact(ttc, batch_mode):
    pairs, want = [], []
    for p in range(12):
        r = 2 + p % 5
        s = C.TTShape([3, 5, 4, 2], [1, r, 3, r + 1, 1])
        x = C.gen_int_tt_np(500 + p, 1, s)
        y = C.gen_int_tt_np(500 + p, 2, s)
        xg, _ = to_gpu(x, "bf16")
        yg, _ = to_gpu(y, "bf16")
        pairs.append((xg, yg))
        want.append(_oracle_pair(x, y))
    plan = ttc.BatchPlan(pairs)
    inner, junc = plan.run()
    for p, (z, K) in enumerate(want):
        assert float(inner[p]) == z
        assert np.array_equal(to_np(plan.junction(junc, p)), K)


_B4096 = {}


def _batch4096(dtype):
    """The 4096-pair batch on the GPU and the oracle's results for every
    pair, cached per dtype: {"held": ...} from the values the GPU holds
    (arithmetic error), and for BF16 also {"unrounded": ...} from the FP64
    values before rounding (total error).  Each entry is (z, K, nx, ny): the
    inner products, junctions V_{N-2} and the two Frobenius norms, all from
    the oracle's right-to-left sweep (V_0 is <X, Y>)."""
    if dtype in _B4096:
        return _B4096[dtype]
    import torch
    shapes = C.batch_pair_shapes(C.SEED_BATCH, 4096)
    td = torch.float32 if dtype == "f32" else torch.bfloat16
    pairs = C.gen_batch_torch(C.SEED_BATCH, shapes, "cuda", td)
    refs = {}
    for name in (("held", "unrounded") if dtype == "bf16" else ("held",)):
        src = pairs if name == "held" else C.gen_batch_torch(C.SEED_BATCH, shapes, "cuda", torch.float64)
        n = len(shapes)
        z, nx, ny, K = np.zeros(n), np.zeros(n), np.zeros(n), []
        for p in range(n):
            x = [to_np(t) for t in src[p][0]]
            y = [to_np(t) for t in src[p][1]]
            V = O.sweep_rl(x, y)
            z[p] = V[0][0, 0]
            K.append(V[len(x) - 2])
            nx[p], ny[p] = tt_norm(x), tt_norm(y)
        refs[name] = (z, K, nx, ny)
        del src
    torch.cuda.empty_cache()
    _B4096[dtype] = (shapes, pairs, refs)
    return _B4096[dtype]


def _check_all(plan, inner, junc, ref, tol):
    """Every pair's inner product (Cauchy-Schwarz scale) and junction
    (rel_err) against the oracle; returns the worst of each."""
    z, K, nx, ny = ref
    e = np.abs(inner - z) / np.maximum(nx * ny, 1e-300)
    bad = np.flatnonzero(e > tol)
    assert bad.size == 0, (bad[:10], e[bad[:10]])
    ek = np.array([rel_err(to_np(plan.junction(junc, p)), K[p]) for p in range(len(K))])
    bad = np.flatnonzero(ek > tol)
    assert bad.size == 0, (bad[:10], ek[bad[:10]])
    return float(e.max()), float(ek.max())


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_batch4096_all_pairs(ttc, dtype, batch_mode):
    """The 4096-pair batch, every pair's inner product and junction against
    the oracle (FP32: on the values the GPU holds; BF16: the total error
    against the unrounded FP64 values and the arithmetic error against the
    rounded ones), then run-to-run determinism bit for bit."""
    _skip_f32_only_bf16(batch_mode, dtype)
    import torch
    shapes, pairs, refs = _batch4096(dtype)
    plan = ttc.BatchPlan(pairs)
    assert plan.config["mode"] == batch_mode
    inner, junc = plan.run()
    inner_np, junc_h = to_np(inner), junc.cpu()
    if dtype == "f32":
        worst = _check_all(plan, inner_np, junc_h, refs["held"], TOL["f32"])
    else:
        worst = _check_all(plan, inner_np, junc_h, refs["unrounded"], TOL["bf16"])
        worst += _check_all(plan, inner_np, junc_h, refs["held"], ARITH_BF16.get(batch_mode, ARITH_BF16_DEFAULT))
    print(f"batch4096 {dtype} {batch_mode}: worst errors {worst}")
    inner2, junc2 = plan.outputs()
    plan.run(inner2, junc2)
    assert np.array_equal(to_np(inner2), inner_np)
    assert torch.equal(junc2, junc)


def test_batch_graph_replays_many_outputs(ttc):
    """Runs into six output-buffer pairs, twice round, queued on the null
    stream with no host synchronisation in between: each new pair captures a
    graph and, past four, evicts the least recently used one while earlier
    replays may still be queued.  Every run equals the first bit for bit."""
    import torch
    shapes = C.batch_pair_shapes(C.SEED_BATCH + 3, 24)
    gpu = []
    for p, (sx, sy) in enumerate(shapes):
        xg, _ = to_gpu(C.gen_tt_np(C.SEED_BATCH + 3, 1 + 2 * p, sx), "f32")
        yg, _ = to_gpu(C.gen_tt_np(C.SEED_BATCH + 3, 2 + 2 * p, sy), "f32")
        gpu.append((xg, yg))
    plan = ttc.BatchPlan(gpu)
    inner0, junc0 = plan.run()
    bufs = [plan.outputs() for _ in range(6)]
    for b in bufs:
        b[0].fill_(float("nan"))
        b[1].fill_(float("nan"))
    outs = []
    for r in range(2):
        for inner, junc in bufs:
            plan.run(inner, junc)
            outs.append((inner.clone(), junc.clone()))
    torch.cuda.synchronize()
    for inner, junc in outs:
        assert torch.equal(inner, inner0) and torch.equal(junc, junc0)


def test_batch_traced_run(ttc):
    """The traced launch gives the untraced results bit for bit; every pair
    has an end clock after its start, its steps' clocks in between and in
    order, and a workgroup inside the plan's grid."""
    shapes = C.batch_pair_shapes(C.SEED_BATCH, 64)
    gpu = []
    for p, (sx, sy) in enumerate(shapes):
        xg, _ = to_gpu(C.gen_tt_np(C.SEED_BATCH, 1 + 2 * p, sx), "f32")
        yg, _ = to_gpu(C.gen_tt_np(C.SEED_BATCH, 2 + 2 * p, sy), "f32")
        gpu.append((xg, yg))
    plan = ttc.BatchPlan(gpu)
    assert plan.config["mode"] in ("lds", "lds1", "persistent", "levels")
    inner, junc = plan.run()
    if plan.config["mode"] not in ("lds", "lds1"):
        pytest.skip("tracing covers the LDS-resident schedules")
    i2, j2, clk, steps = plan.run_traced()
    import torch
    assert torch.equal(i2, inner) and torch.equal(j2, junc)
    clk, steps = clk.numpy(), steps.numpy()
    assert np.all(clk[:, 1] > clk[:, 0])
    assert np.all((clk[:, 2] >= 0) & (clk[:, 2] < 256 * plan.config["wg_per_cu"]))
    for p, (sx, _) in enumerate(shapes):
        s = steps[p, :sx.order]
        assert s[0] >= clk[p, 0] and np.all(np.diff(s) >= 0) and s[-1] == clk[p, 1]


def _abs_sweep_bound(x, y):
    """Largest interface or per-index product of the right-to-left sweep of
    the entrywise absolute values: a bound on every partial sum the GPU
    forms for these cores, whatever its summation order."""
    V, b = np.ones((1, 1)), 1.0
    for k in range(len(x) - 1, 0, -1):
        ax, ay = np.abs(x[k]), np.abs(y[k])
        out = np.zeros((ax.shape[0], ay.shape[0]))
        for i in range(ax.shape[1]):
            b = max(b, float(np.max(ax[:, i, :] @ V)), float(np.max(V @ ay[:, i, :].T)))
            out += ax[:, i, :] @ V @ ay[:, i, :].T
        V = out
        b = max(b, float(np.max(V)))
    return b


@pytest.mark.parametrize("mode", ["lds1b", "lds1"])
def test_batch_bf16_odd_modes_wide_ranks(ttc, monkeypatch, mode):
    """BF16 cores with odd mode sizes (rows starting at odd element offsets,
    so the per-lane funnel shifts differ), ranks up to 128 and G_B wider
    than 32 rows (the BF16-MFMA schedule stages those blocks in LDS): the
    arithmetic-only error against the oracle on the rounded values, and
    exact results for integer cores at the same shapes."""
    monkeypatch.setenv("TTC_BATCH_MODE", mode)
    specs = [([3, 5, 7], [1, 37, 43, 1], [1, 88, 27, 1]),
             ([7, 9, 3, 5], [1, 70, 128, 33, 1], [1, 128, 65, 41, 1]),
             ([5, 11, 7], [1, 100, 47, 1], [1, 33, 120, 1]),
             ([9, 3, 5, 3, 7], [1, 49, 64, 96, 80, 1], [1, 50, 64, 97, 48, 1])]
    gpu, seen = [], []
    for p, (modes, rx, ry) in enumerate(specs):
        xg, xs = to_gpu(C.gen_tt_np(C.SEED_BATCH, 9001 + 2 * p, C.TTShape(modes, rx)), "bf16")
        yg, ys = to_gpu(C.gen_tt_np(C.SEED_BATCH, 9002 + 2 * p, C.TTShape(modes, ry)), "bf16")
        gpu.append((xg, yg))
        seen.append((xs, ys))
    plan = ttc.BatchPlan(gpu)
    assert plan.config["mode"] == mode
    inner, junc = plan.run()
    _check_pairs(plan, to_np(inner), junc, seen, range(len(specs)), ARITH_BF16.get(mode, ARITH_BF16_DEFAULT))
    # integer cores (odd modes, G_B wider than 32 rows): every partial sum of
    # every step is bounded by the sweep of the absolute values, which stays
    # below 2^16, so the 16-bit interface and FP32 sums are exact
    int_specs = [([3, 5, 7], [1, 37, 43, 1], [1, 88, 27, 1]),
                 ([3, 3, 5], [1, 40, 50, 1], [1, 100, 36, 1]),
                 ([3, 5, 3], [1, 128, 33, 1], [1, 70, 49, 1])]
    gpu, want = [], []
    for p, (modes, rx, ry) in enumerate(int_specs):
        x = C.gen_int_tt_np(710 + p, 1, C.TTShape(modes, rx))
        y = C.gen_int_tt_np(710 + p, 2, C.TTShape(modes, ry))
        bound = _abs_sweep_bound(x, y)
        assert bound < 2 ** 16, (p, bound)
        gpu.append((to_gpu(x, "bf16")[0], to_gpu(y, "bf16")[0]))
        want.append(_oracle_pair(x, y))
    plan = ttc.BatchPlan(gpu)
    inner, junc = plan.run()
    for p, (z, K) in enumerate(want):
        assert float(inner[p]) == z
        assert np.array_equal(to_np(plan.junction(junc, p)), K)


def test_batch_plans_from_host_threads(ttc, tmp_path, monkeypatch):
    """Two host threads each build a plan for a batch of their own (FP32 and
    BF16 cores) and run it on a stream of their own at the same time,
    alternating two output buffers so that every run captures a new graph.
    Each result equals the same batch run alone, bit for bit.  The tuner's
    cache file, written by the runs alone, gives the threads' plans the same
    schedule (without it each plan is timed again, under the other thread's
    load)."""
    import threading

    import torch

    monkeypatch.setenv("TTC_AUTOTUNE_CACHE", str(tmp_path / "tune.txt"))
    batches = []
    for n, dtype in enumerate(("f32", "bf16")):
        seed = C.SEED_BATCH + 11 + n
        gpu = []
        for p, (sx, sy) in enumerate(C.batch_pair_shapes(seed, 24)):
            xg, _ = to_gpu(C.gen_tt_np(seed, 1 + 2 * p, sx), dtype)
            yg, _ = to_gpu(C.gen_tt_np(seed, 2 + 2 * p, sy), dtype)
            gpu.append((xg, yg))
        plan = ttc.BatchPlan(gpu)
        inner, junc = plan.run()
        batches.append((gpu, plan.config, to_np(inner), to_np(junc)))
    torch.cuda.synchronize()
    reps = 6
    got = [None] * len(batches)
    errors = []
    start = threading.Barrier(len(batches))

    def work(n):
        try:
            gpu = batches[n][0]
            s = torch.cuda.Stream()
            start.wait()
            with torch.cuda.stream(s):
                plan = ttc.BatchPlan(gpu)
                bufs = [plan.outputs(), plan.outputs()]
                outs = []
                for r in range(reps):
                    inner, junc = bufs[r % 2]
                    plan.run(inner, junc)
                    outs.append((inner.clone(), junc.clone()))
            s.synchronize()
            got[n] = (plan.config, [(to_np(i), to_np(j)) for i, j in outs])
        except Exception as exc:  # re-raised in the main thread
            errors.append(exc)

    threads = [threading.Thread(target=work, args=(n,)) for n in range(len(batches))]
    for t in threads:
        t.start()
    for t in threads:
        t.join(timeout=120)
    assert not any(t.is_alive() for t in threads)
    if errors:
        raise errors[0]
    for n, (_, config, inner0, junc0) in enumerate(batches):
        cfg, outs = got[n]
        assert cfg == config
        for inner, junc in outs:
            assert np.array_equal(inner, inner0) and np.array_equal(junc, junc0), n


@pytest.mark.parametrize("prec", ["bf16", "f32"])
def test_batch_plan_precision(ttc, prec, monkeypatch):
    """The plan's precision selects the step arithmetic for BF16 cores: BF16
    runs the BF16-MFMA schedule, F32 one of the FP32-MFMA schedules, each
    within its bound against the oracle (total and arithmetic-only); BF16
    on FP32 cores is refused."""
    monkeypatch.delenv("TTC_BATCH_MODE", raising=False)
    monkeypatch.delenv("TTC_AUTOTUNE_CACHE", raising=False)
    shapes = C.batch_pair_shapes(C.SEED_BATCH + 7, 24)
    cores64, seen, gpu = [], [], []
    for p, (sx, sy) in enumerate(shapes):
        x = C.gen_tt_np(C.SEED_BATCH + 7, 1 + 2 * p, sx)
        y = C.gen_tt_np(C.SEED_BATCH + 7, 2 + 2 * p, sy)
        xg, xs = to_gpu(x, "bf16")
        yg, ys = to_gpu(y, "bf16")
        cores64.append((x, y))
        seen.append((xs, ys))
        gpu.append((xg, yg))
    plan = ttc.BatchPlan(gpu, prec=prec)
    if prec == "bf16":
        assert plan.config["mode"] == "lds1b"
    else:
        assert plan.config["mode"] != "lds1b"
    inner, junc = plan.run()
    inner = to_np(inner)
    idx = range(len(shapes))
    _check_pairs(plan, inner, junc, cores64, idx, TOL["bf16"])
    _check_pairs(plan, inner, junc, seen, idx, ARITH_BF16["lds1b"] if prec == "bf16" else ARITH_BF16_DEFAULT)
    xf = [to_gpu(x, "f32")[0] for x, _ in cores64[:2]]
    yf = [to_gpu(y, "f32")[0] for _, y in cores64[:2]]
    with pytest.raises(ttc.TTCError) as ei:
        ttc.BatchPlan(list(zip(xf, yf)), prec="bf16")
    assert ei.value.name == "TTC_ERR_UNSUPPORTED"
