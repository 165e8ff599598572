"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for bit.

All arithmetic of the path is integer, so spins, magnetisation, tracked cut and
the per-sweep traces must be identical to the oracle's for every workload,
launch shape and balance mode.
"""
import time

import numpy as np
import pytest

import gdi_synth as gs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gdi():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_00210_amd as gdi

    gdi.lib()
    return gdi


def run_both(gdi, oracle_lib, g, T, seed=1, mode=0, tune=None, trace=True, replica=0, A=1, B=1,
             start_sweep=0, init=None, label="", rule=0):
    print(f"[case] {label} n={g.n} nnz={g.nnz} S={T.size} mode={mode} tune={tune} seed={seed} rule={rule}",
          flush=True)
    ref = oracle_lib.anneal(g, T, seed, A=A, B=B, mode=mode, trace=trace, replica=replica,
                            start_sweep=start_sweep, init=init, rule=rule)
    with gdi.Annealer(g) as a:
        if tune:
            a.tune(**tune)
        r = a.anneal(T, seed, mode=mode, trace=trace, replica=replica, A=A, B=B,
                     start_sweep=start_sweep, init=init, acceptance=rule)
        cw, ce, m = a.cut(r["spins"])
    return ref, r, (cw, ce, m)


def assert_same(ref, r, trace=True, t0=0):
    assert np.array_equal(r["spins"], ref["spins"])
    assert r["M"] == ref["M"]
    assert r["cut"] == ref["cut"]
    if trace:
        assert np.array_equal(r["trace_m"][t0:], ref["trace_m"][t0:])
        assert np.array_equal(r["trace_cut"][t0:], ref["trace_cut"][t0:])


SMALL = {
    "er301_pm1": lambda: gs.er_graph(301, 0.05, 7, "pm1"),
    "rgg2500": lambda: gs.rgg_graph(2500, 8.0, 8, "unit"),
    "torus13": lambda: gs.torus_graph(13, 9, "pm1"),
}


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("mode", [0, 1])
@pytest.mark.parametrize("scope", [1, 2, 3])
def test_small_graphs(gdi, oracle_lib, name, mode, scope):
    g = SMALL[name]()
    T = gs.geometric_temps(2.5, 0.05, 40)
    ref, r, (cw, ce, m) = run_both(gdi, oracle_lib, g, T, seed=11, mode=mode, tune=dict(scope=scope),
                                   label=name)
    assert_same(ref, r)
    assert (cw, m) == (ref["cut"], ref["M"])
    assert ce == oracle_lib.cut(g, ref["spins"])[1]


@pytest.mark.parametrize("tune", [
    dict(scope=1, lanes_per_node=1, block=64),
    dict(scope=1, lanes_per_node=4, block=256),
    dict(scope=1, lanes_per_node=64, block=1024),
    dict(scope=1, lanes_per_node=1, block=256, csr_lds=-1),
    dict(scope=2, grid=8, block=256),
    dict(scope=2, grid=64, block=512),
    dict(scope=2, grid=256, block=1024),
    dict(scope=2, grid=512, block=256),
    dict(scope=2, grid=256, tail_max=-1),
    dict(scope=2, grid=64, tail_max=100),
    dict(scope=2, grid=16, block=512, tail_max=300),
    dict(scope=2, grid=16, leaders=1),
    dict(scope=2, grid=64, leaders=-1),
    dict(scope=2, grid=256, leaders=1, tail_max=-1),
    dict(scope=3, lanes_per_node=1, block=64, grid=1),
    dict(scope=3, lanes_per_node=2, block=128, grid=7),
    dict(scope=3, lanes_per_node=16, block=512, grid=64),
    dict(scope=3, lanes_per_node=8, block=1024, grid=256),
    dict(scope=3, lanes_per_node=32, block=256, grid=300),
])
def test_launch_shape_invariance(gdi, oracle_lib, tune):
    """Same trajectory for every scope, block, grid and lanes-per-node choice (ragged tails)."""
    g = gs.rgg_graph(7777, 10.0, 12, "pm1")
    T = gs.geometric_temps(3.0, 0.05, 30)
    ref, r, _ = run_both(gdi, oracle_lib, g, T, seed=5, tune=tune, label="shape")
    assert_same(ref, r)


@pytest.mark.parametrize("tune", [
    dict(scope=1, lanes_per_node=1, block=256, csr_lds=1),
    dict(scope=1, lanes_per_node=2, block=512, csr_lds=1),
    dict(scope=1, lanes_per_node=8, block=1024, csr_lds=1),
    dict(scope=1, lanes_per_node=64, block=1024, csr_lds=1),
])
def test_lds_resident_launch_shapes(gdi, oracle_lib, tune):
    """The LDS-resident workgroup sweep over lanes-per-node and block choices on a graph
    that fits its 16-bit CSR (3001 nodes, ragged class tails)."""
    g = gs.rgg_graph(3001, 10.0, 13, "pm1")
    assert g.row_ptr[-1] <= 65535
    T = gs.geometric_temps(3.0, 0.05, 30)
    ref, r, _ = run_both(gdi, oracle_lib, g, T, seed=5, tune=tune, label="lds-shape")
    assert_same(ref, r)


@pytest.mark.parametrize("name", ["er800", "torus100"])
def test_small_configs_take_the_lds_resident_sweep(gdi, oracle_lib, name):
    """On one workgroup, er800 and torus100 (+-1 / unit weights, small) run with the whole
    graph in LDS; the same schedule with the CSR in global memory, and the automatic
    choice (one workgroup for er800, the halo grid sweep for the 10,000-node torus), give
    the same result."""
    g, T = gs.workload(name)
    T = T[:300]
    with gdi.Annealer(g) as a:
        r_auto = a.anneal(T, 3, trace=True)
        assert r_auto["result"]["scope"] == (gdi.SCOPE_WORKGROUP if g.n <= 6000 else gdi.SCOPE_GRID)
        a.tune(scope=gdi.SCOPE_WORKGROUP)
        r_lds = a.anneal(T, 3, trace=True)
        a.tune(scope=gdi.SCOPE_WORKGROUP, csr_lds=-1)
        r_glb = a.anneal(T, 3, trace=True)
    assert np.array_equal(r_auto["spins"], r_lds["spins"]) and r_auto["cut"] == r_lds["cut"]
    print(f"{name}: LDS-resident {r_lds['result']['sweep_ms']:.2f} ms, global CSR {r_glb['result']['sweep_ms']:.2f} ms",
          flush=True)
    assert np.array_equal(r_lds["spins"], r_glb["spins"]) and r_lds["cut"] == r_glb["cut"]
    assert np.array_equal(r_lds["trace_cut"], r_glb["trace_cut"])


def test_lds_resident_sweep_rejects_what_does_not_fit(gdi):
    """Weights other than +-1 keep the CSR in global memory; requiring LDS is an error."""
    g = gs.er_graph(400, 0.05, 9, "unit")
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    up = g.col > rows
    heavy = gs.from_edges(g.n, rows[up], g.col[up], np.full(int(up.sum()), 2))
    with gdi.Annealer(heavy) as a:
        a.tune(scope=1, csr_lds=1)
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(np.ones(2), 1)
        assert e.value.code == gdi.ERANGE
    big = gs.rgg_graph(7777, 10.0, 12, "pm1")  # nnz beyond the 16-bit row pointers
    assert big.row_ptr[-1] > 65535
    with gdi.Annealer(big) as a:
        a.tune(scope=1, csr_lds=1)
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(np.ones(2), 1)
        assert e.value.code == gdi.ERANGE
        a.tune(scope=1, csr_lds=0)  # the automatic choice falls back to the global CSR
        a.anneal(np.ones(2), 1)


def test_er800_full_schedule(gdi, oracle_lib):
    g, T = gs.workload("er800")
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="er800")
    assert_same(ref, r)


def test_torus100_full_schedule(gdi, oracle_lib):
    g, T = gs.workload("torus100")
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="torus100")
    assert_same(ref, r)
    assert r["M"] == 0


def test_rgg1m_full_schedule_bench_launch(gdi, oracle_lib):
    """The benchmark workload and launch configuration, all 2000 sweeps, traces included."""
    g, T = gs.workload("rgg1m")
    t = time.time()
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="rgg1m")
    print(f"rgg1m: both sides in {time.time() - t:.1f}s, GPU sweep {r['result']['sweep_ms']:.1f} ms",
          flush=True)
    assert r["result"]["scope"] == gdi.SCOPE_GRID
    assert_same(ref, r)


def test_rgg1m_fenced_grid_path(gdi, oracle_lib):
    """The fenced grid sweep (global gathers) on the same graph, first 300 sweeps."""
    g, T = gs.workload("rgg1m")
    T = T[:300]
    ref, r, _ = run_both(gdi, oracle_lib, g, T, tune=dict(scope=3), label="rgg1m-fenced")
    assert_same(ref, r)


def test_rgg8m_sanity_run_bench_launch(gdi, oracle_lib):
    """The 8M-node RGG (working set above the on-package cache), its whole 50-sweep
    schedule in the launch configuration the benchmark uses, traces included."""
    g, T = gs.workload("rgg8m")
    t = time.time()
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="rgg8m")
    print(f"rgg8m: both sides in {time.time() - t:.1f}s, GPU sweep {r['result']['sweep_ms']:.1f} ms",
          flush=True)
    assert r["result"]["scope"] == gdi.SCOPE_GRID
    assert_same(ref, r)


def test_general_weight_form_on_unit_weights(gdi, oracle_lib):
    """The halo sweep's general-weight form forced on a unit-weight graph: same results."""
    g = gs.rgg_graph(150_000, 8.0, 44, "unit")
    T = gs.geometric_temps(3.0, 0.05, 120)
    ref, r, _ = run_both(gdi, oracle_lib, g, T, tune=dict(general_weights=1), label="general-weights")
    assert r["result"]["scope"] == gdi.SCOPE_GRID
    assert_same(ref, r)


def test_halo_thresholds_from_global_memory(gdi, oracle_lib):
    """Temperatures high enough that the threshold row is wider than the LDS copy the
    halo sweep keeps (K > 4096): the thresholds are then read from global memory."""
    g = gs.rgg_graph(90_000, 8.0, 45, "pm1")
    T = gs.geometric_temps(400.0, 0.5, 30)
    assert int(np.floor(32 * np.log(2) * T.max())) > 4096
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="global-thresholds")
    assert r["result"]["scope"] == gdi.SCOPE_GRID and r["result"]["table_width"] > 4096
    assert_same(ref, r)


def test_odd_n_negative_weights_and_coefficients(gdi, oracle_lib):
    g = gs.er_graph(999, 0.01, 13, "pm1")
    T = gs.geometric_temps(4.0, 0.1, 50)
    for A, B in ((3, 2), (0, 1), (1, 0), (2, -1)):
        ref, r, _ = run_both(gdi, oracle_lib, g, T, A=A, B=B, label=f"A{A}B{B}")
        assert_same(ref, r)


def test_degenerate_graphs(gdi, oracle_lib):
    T = gs.geometric_temps(2.0, 0.05, 20)
    # two nodes, one edge
    g = gs.from_edges(2, [0], [1], [1])
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="k2")
    assert_same(ref, r)
    # no edges at all: one colour class
    g = gs.Graph(n=65, row_ptr=np.zeros(66, np.int32), col=np.zeros(0, np.int32),
                 w=np.zeros(0, np.int32), name="empty")
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="no-edges")
    assert_same(ref, r)
    # a star: one row of 4000 entries, 4000 rows of one entry; isolated nodes too
    a = np.zeros(4000, np.int64); b = np.arange(1, 4001)
    g = gs.from_edges(4100, a, b, np.ones(4000, np.int64))
    for scope in (1, 2, 3):
        ref, r, _ = run_both(gdi, oracle_lib, g, T, tune=dict(scope=scope), label="star")
        assert_same(ref, r)
    # a hub row too long for the grid sweep's LDS overflow region (50,000 entries): the
    # sweep reads the entries past the first 16 from memory instead
    a = np.zeros(50000, np.int64); b = np.arange(1, 50001)
    g = gs.from_edges(50001, a, b, np.ones(50000, np.int64))
    ref, r, _ = run_both(gdi, oracle_lib, g, T, tune=dict(scope=2), label="big star")
    assert_same(ref, r)


PAPER_PF = gs.geometric_temps(0.2, 0.001, 60)


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("rule", [0, 1])
def test_redundant_tail(gdi, oracle_lib, name, rule):
    """The grid sweep's redundant tail (the last classes, run by every workgroup with
    workgroup barriers only) follows the oracle's trajectory under both rules."""
    g = SMALL[name]()
    T = gs.geometric_temps(2.5, 0.05, 40) if rule == 0 else PAPER_PF[:40]
    ref, r, _ = run_both(gdi, oracle_lib, g, T, seed=13, tune=dict(scope=2, tail_max=960), label=f"tail {name}",
                         rule=rule)
    assert_same(ref, r)


@pytest.mark.parametrize("scope", [1, 2, 3])
@pytest.mark.parametrize("mode", [0, 1])
def test_paper_rule(gdi, oracle_lib, scope, mode):
    """The paper's acceptance rule: argmin value, then a random flip with probability P_f."""
    g = gs.rgg_graph(9000, 8.0, 23, "pm1")
    ref, r, _ = run_both(gdi, oracle_lib, g, PAPER_PF, seed=4, mode=mode, tune=dict(scope=scope), rule=1,
                         label="paper-rule")
    assert_same(ref, r)


def test_paper_rule_on_the_1m_graph(gdi, oracle_lib):
    g, _ = gs.workload("rgg1m")
    pf = gs.geometric_temps(0.2, 0.001, 200)
    ref, r, _ = run_both(gdi, oracle_lib, g, pf, rule=1, label="paper-rule-rgg1m")
    assert r["result"]["scope"] == gdi.SCOPE_GRID
    assert_same(ref, r)


def test_paper_rule_batched(gdi, oracle_lib):
    graphs = [gs.er_graph(900, 0.03, 24), gs.rgg_graph(3000, 12.0, 25, "pm1")]
    anns = [gdi.Annealer(g) for g in graphs]
    items = [(anns[0].h, graphs[0].n, 0), (anns[1].h, graphs[1].n, 0), (anns[1].h, graphs[1].n, 3)]
    out = gdi.anneal_batch(items, PAPER_PF, 8, acceptance=1)
    for i, (g, rep) in enumerate(((graphs[0], 0), (graphs[1], 0), (graphs[1], 3))):
        ref = oracle_lib.anneal(g, PAPER_PF, 8, replica=rep, rule=1)
        assert np.array_equal(out["spins"][i], ref["spins"]) and out["cut"][i] == ref["cut"]
    for a in anns:
        a.close()


def test_paper_rule_rejects_bad_probabilities(gdi):
    g = gs.er_graph(100, 0.05, 26)
    with gdi.Annealer(g) as a:
        for bad in (np.array([0.5, 1.5]), np.array([-0.1]), np.array([np.nan])):
            with pytest.raises(gdi.GdiError) as e:
                a.anneal(bad, 1, acceptance=1)
            assert e.value.code == gdi.EINVAL
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(np.ones(3), 1, acceptance=2)
        assert e.value.code == gdi.EINVAL
        r = a.anneal(np.full(3, 0.5), 1, acceptance=1)
        assert r["spins"].shape == (g.n,)


@pytest.mark.parametrize("mode,rule", [(0, 0), (1, 0), (0, 1)])
def test_standard_solver_dense_balance(gdi, oracle_lib, mode, rule):
    """Alg. 2's dense balance term (every decision sums all n spins) gives the tracked
    sweep's results bit for bit."""
    g = gs.rgg_graph(6000, 8.0, 27, "pm1")
    T = PAPER_PF[:30] if rule else gs.geometric_temps(3.0, 0.05, 30)
    print(f"[case] dense balance mode={mode} rule={rule}", flush=True)
    ref = oracle_lib.anneal(g, T, 2, mode=mode, rule=rule, trace=True)
    with gdi.Annealer(g) as a:
        r = a.anneal(T, 2, mode=mode, acceptance=rule, flags=gdi.FLAG_DENSE_BALANCE, trace=True)
    assert_same(ref, r)


def test_standard_solver_needs_one_workgroup(gdi):
    g = gs.rgg_graph(70_000, 8.0, 28)
    with gdi.Annealer(g) as a:
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(np.ones(2), 1, flags=gdi.FLAG_DENSE_BALANCE)
        assert e.value.code == gdi.ERANGE
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(np.ones(2), 1, flags=8)
        assert e.value.code == gdi.EINVAL


@pytest.mark.parametrize("grid", [0, 8])
def test_asynchronous_sweep_against_the_oracle(gdi, oracle_lib, grid):
    """Alg. 3 as printed is racy and not reproducible; what must hold: the global G that
    only the per-flip atomic adds maintained equals the magnetisation of the returned
    spins as the oracle counts it, and the returned cut is the oracle's cut of those
    spins (Sec. V-C: the atomic adds keep G valid at the end of each sweep)."""
    g = gs.rgg_graph(100_000, 8.0, 29)
    T = gs.geometric_temps(3.0, 0.05, 300)
    rand = oracle_lib.cut(g, oracle_lib.anneal(g, T[:1], 3, start_sweep=1)["spins"])[0]
    print(f"[case] asynchronous sweep grid={grid}", flush=True)
    with gdi.Annealer(g) as a:
        det = a.anneal(T, 3)
        a.tune(grid=grid)
        for rule, temps in ((gdi.ACCEPT_METROPOLIS, T), (gdi.ACCEPT_PAPER, gs.geometric_temps(0.05, 1e-4, 300))):
            rac = a.anneal(temps, 3, flags=gdi.FLAG_RACY, acceptance=rule)
            cw, ce, m = oracle_lib.cut(g, rac["spins"])
            print(f"rule {rule}: deterministic cut {det['cut']} M {det['M']}; asynchronous cut {rac['cut']} "
                  f"M {rac['M']} (grid {rac['result']['grid']}); random state cut {rand}", flush=True)
            assert (cw, m) == (rac["cut"], rac["M"])
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(T, 3, flags=gdi.FLAG_RACY, trace=True)
        assert e.value.code == gdi.EINVAL


def test_large_weights_mid_size_fall_back_to_one_workgroup(gdi, oracle_lib):
    """A 20,000-node graph would take the halo sweep, but its weights exceed the packed
    range: the automatic choice runs it on one workgroup instead."""
    g0 = gs.rgg_graph(20_000, 8.0, 23)
    rows = np.repeat(np.arange(g0.n), np.diff(g0.row_ptr))
    up = g0.col > rows
    rng = np.random.default_rng(4)
    w = rng.integers(-3000, 3001, int(up.sum()))
    w[w == 0] = 1
    g = gs.from_edges(g0.n, rows[up], g0.col[up], w)
    T = gs.geometric_temps(4000.0, 50.0, 30)
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="heavy-mid")
    assert r["result"]["scope"] == gdi.SCOPE_WORKGROUP
    assert_same(ref, r)


def test_large_weights_take_the_fenced_grid_sweep(gdi, oracle_lib):
    """The halo sweep packs weights into 11 bits; heavier graphs run the fenced grid sweep."""
    g0 = gs.rgg_graph(70_000, 8.0, 22)
    rows = np.repeat(np.arange(g0.n), np.diff(g0.row_ptr))
    up = g0.col > rows
    rng = np.random.default_rng(3)
    w = rng.integers(-3000, 3001, int(up.sum()))
    w[w == 0] = 1
    g = gs.from_edges(g0.n, rows[up], g0.col[up], w)
    T = gs.geometric_temps(4000.0, 50.0, 20)
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="heavy")
    assert r["result"]["scope"] == gdi.SCOPE_GRID_FENCED
    assert_same(ref, r)
    with gdi.Annealer(g) as a:
        a.tune(scope=2)
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(T, 1)
        assert e.value.code == gdi.ERANGE


def test_single_sweep_and_empty_resume(gdi, oracle_lib):
    g = gs.rgg_graph(3000, 8.0, 14)
    T = gs.geometric_temps(2.0, 0.05, 1)
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="S=1")
    assert_same(ref, r)
    # start_sweep == S: nothing runs, the initial state comes back
    init = np.where(np.arange(g.n) % 3 == 0, 1, -1).astype(np.int8)
    ref, r, _ = run_both(gdi, oracle_lib, g, T, start_sweep=1, init=init, trace=False, label="S=0")
    assert np.array_equal(r["spins"], init) and np.array_equal(ref["spins"], init)


def test_infinite_temperature_alternation(gdi, oracle_lib):
    g = gs.er_graph(400, 0.03, 15, "pm1")
    T = np.full(9, 1e300)
    ref, r, _ = run_both(gdi, oracle_lib, g, T, label="T=inf")
    assert_same(ref, r)


def test_resume_on_gpu(gdi, oracle_lib):
    g = gs.rgg_graph(150_000, 8.0, 16)
    T = gs.geometric_temps(3.0, 0.05, 120)
    with gdi.Annealer(g) as a:
        full = a.anneal(T, 21, trace=True)
        head = a.anneal(T[:50], 21)
        tail = a.anneal(T, 21, start_sweep=50, init=head["spins"], trace=True)
    assert np.array_equal(full["spins"], tail["spins"])
    assert np.array_equal(full["trace_cut"][50:], tail["trace_cut"][50:])
    ref = oracle_lib.anneal(g, T, 21)
    assert np.array_equal(full["spins"], ref["spins"])


def test_replicas_and_repeat_determinism(gdi, oracle_lib):
    g = gs.er_graph(2000, 0.01, 17)
    T = gs.geometric_temps(2.0, 0.05, 60)
    with gdi.Annealer(g) as a:
        outs = [a.anneal(T, 3, replica=rep) for rep in (0, 1, 255, 1)]
    assert np.array_equal(outs[1]["spins"], outs[3]["spins"])
    assert not np.array_equal(outs[0]["spins"], outs[1]["spins"])
    for rep, o in zip((0, 1, 255), outs[:3]):
        ref = oracle_lib.anneal(g, T, 3, replica=rep)
        assert np.array_equal(o["spins"], ref["spins"])


def test_device_pointer_path(gdi, oracle_lib):
    """gdi_anneal_dev / gdi_cut_dev on torch device memory and torch's stream."""
    import torch

    g = gs.rgg_graph(90_000, 8.0, 18, "pm1")
    T = gs.geometric_temps(3.0, 0.05, 80)
    ref = oracle_lib.anneal(g, T, 8)
    out = torch.full((g.n,), 7, dtype=torch.int8, device="cuda:0")
    s = torch.cuda.Stream()
    with torch.cuda.stream(s), gdi.Annealer(g) as a:
        a.set_stream(s.cuda_stream)
        a.anneal_dev(T, 8, out.data_ptr())
        res = a.result()
        cw, ce, m = a.cut_dev(out.data_ptr())
    s.synchronize()
    assert np.array_equal(out.cpu().numpy(), ref["spins"])
    assert (res.magnetization, res.cut_weighted) == (ref["M"], ref["cut"])
    assert (cw, m) == (ref["cut"], ref["M"])


def test_forced_barrier_timeout_reports_error_and_recovers(gdi, oracle_lib):
    """A host-set tiny spin limit makes the bounded barrier waits give up: GDI_ETIMEOUT, no hang."""
    g = gs.rgg_graph(20_000, 8.0, 19)
    T = gs.geometric_temps(3.0, 0.05, 20)
    with gdi.Annealer(g) as a:
        for scope in (2, 3):
            a.tune(scope=scope, grid=256, spin_limit=1)
            with pytest.raises(gdi.GdiError) as e:
                a.anneal(T, 1)
            assert e.value.code == gdi.ETIMEOUT
            a.tune(reset=True)
            a.tune(scope=scope)
            r = a.anneal(T, 1)
            assert np.array_equal(r["spins"], oracle_lib.anneal(g, T, 1)["spins"])


def test_bad_schedule_is_rejected(gdi):
    g = gs.er_graph(100, 0.05, 20)
    with gdi.Annealer(g) as a:
        for T in (np.array([1.0, 0.0]), np.array([np.nan]), np.array([-1.0])):
            with pytest.raises(gdi.GdiError) as e:
                a.anneal(T, 1)
            assert e.value.code == gdi.EINVAL
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(np.ones(3), 1, mode=7)
        assert e.value.code == gdi.EINVAL
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(np.ones(3), 1, A=2**28)
        assert e.value.code == gdi.ERANGE
        r = a.anneal(np.ones(3), 1)  # still usable
        assert r["spins"].shape == (g.n,)


def _star_plus_matching(n, seed):
    """One hub joined to every other node plus a random matching: one very long row,
    many rows of length 1-2 (the cut kernel's lanes per row follow the mean degree)."""
    rng = np.random.default_rng(seed)
    hub_a = np.zeros(n - 1, dtype=np.int64)
    hub_b = np.arange(1, n)
    perm = rng.permutation(np.arange(1, n))
    m_a, m_b = perm[0::2][: (n - 1) // 2], perm[1::2][: (n - 1) // 2]
    a = np.concatenate([hub_a, m_a])
    b = np.concatenate([hub_b, m_b])
    w = rng.choice(np.array([-3, -1, 1, 2]), size=a.size)
    return gs.from_edges(n, a, b, w)


@pytest.mark.parametrize("kind", ["path", "star_matching", "rgg8", "er20", "er70"])
def test_cut_from_scratch_over_row_widths(gdi, oracle_lib, kind):
    """gdi_cut (k_reduce) against the oracle's count on graphs from mean degree 2 (one
    long row among short ones, a path) to 70, i.e. with 2 and 4 lanes per row and rows of
    one to many rounds, on random states; the allocation-free entry point gives the same
    three values."""
    torch = pytest.importorskip("torch")
    n = 3000
    if kind == "path":
        a = np.arange(n - 1)
        g = gs.from_edges(n, a, a + 1, np.where(a % 3 == 0, -2, 1))
    elif kind == "star_matching":
        g = _star_plus_matching(n, 5)
    elif kind == "rgg8":
        g = gs.rgg_graph(n, 8.0, 6, "pm1")
    elif kind == "er20":
        g = gs.er_graph(n, 20.0 / (n - 1), 7, "pm1")
    else:
        g = gs.er_graph(n, 70.0 / (n - 1), 8, "unit")
    rng = np.random.default_rng(9)
    print(f"[case] cut {kind} n={g.n} nnz={g.nnz}", flush=True)
    with gdi.Annealer(g) as a:
        for rep in range(3):
            spins = np.where(rng.random(g.n) < (0.2 + 0.3 * rep), 1, -1).astype(np.int8)
            ref = oracle_lib.cut(g, spins)
            assert tuple(a.cut(spins)) == ref
            d_sp = torch.from_numpy(spins).to("cuda:0")
            d_out = torch.zeros(3, dtype=torch.int64, device="cuda:0")
            a.cut_dev_noalloc(d_sp.data_ptr(), d_out.data_ptr())
            torch.cuda.synchronize()
            assert tuple(int(x) for x in d_out.cpu()) == ref
