"""Batched pressure solves (many cases of different grids, one blocked SOR
launch per sweep over all their tiles): every case's steps are bit for bit
those of the same context stepped alone, whatever the mix of grid sizes, tile
shapes and convergence points."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _cases():
    from paper_2402_17337_amd import workloads as W
    return [W.small_plunging(64, 48), W.stationary_128x96(), W.plunging_stretched(256, 192, 0.05),
            W.small_plunging(96, 64, seed=3)]


def _solver(wl, tile=None, **over):
    from paper_2402_17337_amd import ibm
    s = ibm.Solver(wl["nx"], wl["ny"], wl["xf"], wl["yf"], wl["u0"], wl["v0"], wl["p0"], **dict(wl["params"], **over))
    if tile:
        assert s.set_option(ibm.OPT_TB_TILE_X, tile[0]) == ibm.OK
        assert s.set_option(ibm.OPT_TB_TILE_Y, tile[1]) == ibm.OK
    return s


TILES = [None, (64, 24), None, (32, 16)]


def test_batched_steps_equal_solo_steps_bitwise():
    _need_gpu()
    from paper_2402_17337_amd import ibm
    wls = _cases()
    solo = [_solver(w, t) for w, t in zip(wls, TILES)]
    batched = [_solver(w, t) for w, t in zip(wls, TILES)]
    batch = ibm.Batch(batched)
    for step in range(3):
        st_b = batch.step(1)
        for k, s in enumerate(solo):
            st = s.step(1)
            assert st["rc"] == ibm.OK and st_b[k]["status"] == ibm.OK
            assert st["p_iters"] == st_b[k]["p_iters"], (step, k, st["p_iters"], st_b[k]["p_iters"])
            assert st["p_rel"] == st_b[k]["p_rel"] and st["p_r0"] == st_b[k]["p_r0"]
            assert st["cd"] == st_b[k]["cd"] and st["cl"] == st_b[k]["cl"]
    iters = [st["p_iters"] for st in st_b]
    assert len(set(iters)) > 1  # the cases finish at different iterations
    for a, b in zip(solo, batched):
        for x, y in zip(a.fields(), b.fields()):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("check", [10, 100])
def test_mixed_precision_batch_equals_solo_steps_bitwise(check):
    """FP32 sweeps with FP64 refinement: the batched refinements, sweeps and
    stop tests give every case the steps of its context stepped alone."""
    _need_gpu()
    from paper_2402_17337_amd import ibm
    wls = _cases()
    over = dict(p_method=ibm.RBSOR_MP, p_check=check)
    solo = [_solver(w, t, **over) for w, t in zip(wls, TILES)]
    batch = ibm.Batch([_solver(w, t, **over) for w, t in zip(wls, TILES)])
    for step in range(3):
        st_b = batch.step(1)
        for k, s in enumerate(solo):
            st = s.step(1)
            assert st["rc"] == ibm.OK and st_b[k]["status"] == ibm.OK
            for key in ("p_iters", "p_rel", "p_r0", "cd", "cl"):
                assert st[key] == st_b[k][key], (step, k, key, st[key], st_b[k][key])
    assert len(set(st["p_iters"] for st in st_b)) > 1
    for a, b in zip(solo, batch.solvers):
        for x, y in zip(a.fields(), b.fields()):
            assert np.array_equal(x, y)


@pytest.mark.parametrize("intervals,cap,mixed", [(4, None, False), (6, 1234, False), (4, None, True),
                                                 (6, 1234, True)])
def test_graph_replayed_batch_equals_launched_batch_bitwise(intervals, cap, mixed):
    """Stretches of `intervals` check intervals replayed from one HIP graph,
    with each case's steps around the solve run eagerly between the replays:
    every step equals the batch launched interval by interval.  With the cap
    (1234 iterations: 30 stretches of 40 or 20 of 60, then intervals launched
    one by one, the last of 4 iterations) some solves end at the limit; in
    the uncapped run the cases finish inside stretches.  The last step runs
    with the graph switched off again.  mixed: FP32 sweeps with FP64
    refinement every 10 iterations (the stretch holds the sweeps, the
    refinement and the stop tests of each interval)."""
    _need_gpu()
    from paper_2402_17337_amd import ibm
    wls = _cases()
    over = {} if cap is None else {"p_max_iter": cap}
    if mixed:
        over.update(p_method=ibm.RBSOR_MP, p_check=10)
    plain = ibm.Batch([_solver(w, t, **over) for w, t in zip(wls, TILES)])
    graphed = ibm.Batch([_solver(w, t, **over) for w, t in zip(wls, TILES)])
    graphed.set_graph(intervals)
    for step in range(4):
        if step == 3:
            graphed.set_graph(0)
        st_p, st_g = plain.step(1), graphed.step(1)
        assert st_p[0]["rc"] == st_g[0]["rc"]
        for a, b in zip(st_p, st_g):
            for key in ("status", "p_iters", "p_rel", "p_r0", "cd", "cl"):
                assert a[key] == b[key], (step, key, a[key], b[key])
    iters = [st["p_iters"] for st in st_p]
    if cap is None:
        assert len(set(iters)) > 1 and any(k % (10 * intervals) for k in iters)
    else:
        assert cap in iters
    for a, b in zip(plain.solvers, graphed.solvers):
        for x, y in zip(a.fields(), b.fields()):
            assert np.array_equal(x, y)


def test_batch_validation():
    _need_gpu()
    from paper_2402_17337_amd import ibm
    wls = _cases()
    a = _solver(wls[0])
    p = ibm.Solver(wls[1]["nx"], wls[1]["ny"], wls[1]["xf"], wls[1]["yf"], **dict(wls[1]["params"], p_method=ibm.PCG))
    with pytest.raises(ibm.IbmError):
        ibm.Batch([a, p])           # PCG cannot join
    m = ibm.Solver(wls[1]["nx"], wls[1]["ny"], wls[1]["xf"], wls[1]["yf"],
                   **dict(wls[1]["params"], p_method=ibm.RBSOR_MP))
    with pytest.raises(ibm.IbmError):
        ibm.Batch([a, m])           # one method for all
    with pytest.raises(ibm.IbmError):
        ibm.Batch([a, a])           # a context appears once
    other = torch.cuda.Stream()
    q = ibm.Solver(wls[1]["nx"], wls[1]["ny"], wls[1]["xf"], wls[1]["yf"], stream=other, **wls[1]["params"])
    with pytest.raises(ibm.IbmError):
        ibm.Batch([a, q])           # one stream for all
    b = _solver(wls[2])
    assert b.set_option(ibm.OPT_TB_SWEEPS, 4) == ibm.OK
    with pytest.raises(ibm.IbmError):
        ibm.Batch([a, b])           # one sweep count for all
    batch = ibm.Batch([a])
    for bad in (3, -2, 1002):
        with pytest.raises(ibm.IbmError):
            batch.set_graph(bad)    # even counts from 2 to 1000, or 0
    batch.set_graph(2)
    batch.set_graph(0)


def test_autotune_picks_a_candidate_and_keeps_the_iterates():
    _need_gpu()
    from paper_2402_17337_amd import ibm
    wl = _cases()[2]
    a, b = _solver(wl), _solver(wl)
    best, times = b.autotune_tiles(candidates=((76, 44), (48, 16)), iters=50)
    assert best in times and len(times) == 2 and all(v > 0 for v in times.values())
    for _ in range(2):
        sa, sb = a.step(1), b.step(1)
        assert sa["p_iters"] == sb["p_iters"]
    for x, y in zip(a.fields()[:3], b.fields()[:3]):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("mixed", [False, True])
def test_full_batched_workload_equals_case_by_case_bitwise(mixed):
    """The 64-case workload (grids 256x192 to 1024x768, 21.1 M cells) in the
    benchmark's launch configuration (default 76x44 tiles, solves capped; FP32 sweeps
    refined every 100 iterations for the mixed form): two batched steps equal
    the same contexts stepped one by one, bit for bit, for every case (the
    second step starts from the first one's pressure, so its initial-residual
    sums run over partials of nonzero values on the largest grids)."""
    _need_gpu()
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import workloads as W
    cases = W.batched_plunging(64, 0)
    over = dict(p_max_iter=300)
    if mixed:
        over.update(p_method=ibm.RBSOR_MP, p_check=100)

    def make():
        return [ibm.Solver(c["nx"], c["ny"], c["xf"], c["yf"], c["u0"], c["v0"], c["p0"],
                           **dict(c["params"], **over)) for c in cases]
    solo = make()
    batch = ibm.Batch(make())
    for step in range(2):
        st_b = batch.step(1)
        for k, s in enumerate(solo):
            st = s.step(1)
            for key in ("status", "p_iters", "p_rel", "p_r0", "cd", "cl"):
                assert st[key] == st_b[k][key], (step, k, key, st[key], st_b[k][key])
            if k % 16 == 0:  # fields of a sample of the cases
                for x, y in zip(s.fields(), batch.solvers[k].fields()):
                    assert np.array_equal(x, y)
    batch.close()  # the batch borrows its contexts: release it first
    for s in solo + batch.solvers:
        s.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_full_size_batch_to_tolerance_leaves_the_residual_as_divergence(mixed):
    """The largest case of the 64-case workload (1024x768) and a 512x384 one,
    one batched step to the 1e-8 tolerance, uncapped (FP32 sweeps refined every
    100 iterations for the mixed form): for every case the projection leaves
    V D(u^{n+1}) = dt (V b - A phi) where no mass source acts, and that
    residual meets the stop test (a property that holds at any size; A is the
    oracle's operator)."""
    _need_gpu()
    from oracle import oracle as O
    from paper_2402_17337_amd import ibm
    from paper_2402_17337_amd import workloads as W
    from projection_identity import divergence_identity
    cases = W.batched_plunging(64, 0)
    big = max(cases, key=lambda c: c["nx"] * c["ny"])
    mid = next(c for c in cases if c["nx"] == 512)
    picked = [big, mid]
    over = dict(p_method=ibm.RBSOR_MP, p_check=100) if mixed else {}
    solvers = [ibm.Solver(c["nx"], c["ny"], c["xf"], c["yf"], c["u0"], c["v0"], c["p0"], **dict(c["params"], **over))
               for c in picked]
    batch = ibm.Batch(solvers)
    st = batch.step(1)
    for c, s, sb in zip(picked, solvers, st):
        print(c["name"], "iterations", sb["p_iters"], "p_rel", sb["p_rel"], flush=True)
        assert sb["status"] == ibm.OK and sb["p_rel"] <= c["params"]["p_tol"] and sb["p_iters"] > 10000
        u, v, _, phi = s.fields()
        A = O.Oracle(c["nx"], c["ny"], c["xf"], c["yf"], **c["params"]).apply_A
        d = divergence_identity(u, v, s.poisson_rhs(), phi, s.ibm()["msrc"], c["xf"], c["yf"], c["params"]["dt"], A)
        print("divergence identity", d, flush=True)
        assert d["rel"] <= c["params"]["p_tol"] and abs(d["rel"] - sb["p_rel"]) <= 1e-3 * d["rel"]
        assert d["scale"] > 100 * d["bar"] and d["err"] <= d["bar"]
    batch.close()
    for s in solvers:
        s.close()


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("mixed", [False, True])
def test_batched_steps_match_the_oracle(mixed):
    """Four cases of different grids stepped as one batch against the FP64
    oracle stepping each case alone (Sec. 2.2 time steps, Eqs. 1-4): each case
    replays its oracle iteration counts (the stop test compares a residual
    whose last digits depend on rounding order), and u, v, p agree to the
    FP64 bar of 1e-10 (relative L2).  Mixed form: FP32 sweeps refined every
    100 iterations against the oracle's mixed-precision solve, to the bar of
    the single-grid mixed test (the two sides round the float sweeps
    differently): u, v within 1e-8, p within 1e-6; the distance to the FP64
    oracle is printed."""
    _need_gpu()
    from oracle import oracle as O
    from paper_2402_17337_amd import ibm
    wls = _cases()
    nsteps = 3
    over_o = dict(p_method=O.SOR_MP, p_check=100) if mixed else {}
    over_g = dict(p_method=ibm.RBSOR_MP, p_check=100) if mixed else {}
    orcs, iters = [], []
    for w in wls:
        o = O.Oracle(w["nx"], w["ny"], w["xf"], w["yf"], w["u0"], w["v0"], w["p0"], **dict(w["params"], **over_o))
        rc, so = o.step(nsteps)
        assert rc == O.OK, so
        orcs.append(o)
        iters.append([s["p_iters"] for s in so])
    solvers = [_solver(w, t, **over_g) for w, t in zip(wls, TILES)]
    for s, it in zip(solvers, iters):
        s.set_poisson_schedule(it)
    batch = ibm.Batch(solvers)
    for step in range(nsteps):
        st_b = batch.step(1)
        for k in range(len(wls)):
            assert st_b[k]["status"] == ibm.OK and st_b[k]["p_iters"] == iters[k][step], (step, k, st_b[k])
    for k, (s, o) in enumerate(zip(solvers, orcs)):
        ug, vg, pg, _ = s.fields()
        uo, vo, po, _ = o.fields()
        e = (_rel_l2(ug, uo), _rel_l2(vg, vo), _rel_l2(pg, po))
        print(f"case {k} ({wls[k]['nx']}x{wls[k]['ny']}) iters {iters[k]}: u {e[0]:.2e} v {e[1]:.2e} p {e[2]:.2e}",
              flush=True)
        if mixed:
            assert e[0] <= 1e-8 and e[1] <= 1e-8 and e[2] <= 1e-6, (k, e)
        else:
            assert max(e) <= 1e-10, (k, e)
    assert len({tuple(i) for i in iters}) > 1
    batch.close()
    for s in solvers:
        s.close()


def test_per_case_limits_must_fall_on_check_intervals():
    """A batch advances in whole check intervals: contexts with different
    iteration limits are accepted when every limit is a multiple of the check
    interval (each case then stops at its own limit, bit for bit as when
    stepped alone), and rejected otherwise."""
    _need_gpu()
    from paper_2402_17337_amd import ibm
    wls = _cases()
    with pytest.raises(ibm.IbmError):
        ibm.Batch([_solver(wls[0], p_max_iter=35), _solver(wls[1], p_max_iter=50)])
    limits = [30, 50, 70, 40]
    solo = [_solver(w, t, p_max_iter=m) for w, t, m in zip(wls, TILES, limits)]
    batch = ibm.Batch([_solver(w, t, p_max_iter=m) for w, t, m in zip(wls, TILES, limits)])
    for step in range(2):
        st_b = batch.step(1)
        for k, s in enumerate(solo):
            st = s.step(1)
            assert st["p_iters"] == limits[k] == st_b[k]["p_iters"]
            assert st["rc"] == ibm.NOT_CONVERGED and st_b[k]["status"] == ibm.NOT_CONVERGED
            assert st["p_rel"] == st_b[k]["p_rel"]
    for a, b in zip(solo, batch.solvers):
        for x, y in zip(a.fields(), b.fields()):
            assert np.array_equal(x, y)
    batch.close()
