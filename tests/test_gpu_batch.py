"""GPU parity of the batched form: every instance of one persistent launch equals the
oracle's single run of that (graph, seed, replica), bit for bit, for any launch tuning."""
from concurrent.futures import ThreadPoolExecutor

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


def oracle_runs(oracle_lib, cases, T, seed, mode=0):
    """cases: list of (graph, replica); oracle calls in parallel host threads."""
    def one(c):
        g, rep = c
        return oracle_lib.anneal(g, T, seed, replica=rep, mode=mode, n_threads=1)
    with ThreadPoolExecutor(max_workers=16) as ex:
        return list(ex.map(one, cases))


def make_items(gdi, graphs, replicas_of):
    anns = [gdi.Annealer(g) for g in graphs]
    items, cases = [], []
    for a, g, reps in zip(anns, graphs, replicas_of):
        for r in reps:
            items.append((a.h, g.n, r))
            cases.append((g, r))
    return anns, items, cases


MIXED = [
    lambda: gs.er_graph(900, 0.03, 71, "unit"),
    lambda: gs.rgg_graph(3000, 12.0, 72, "pm1"),
    lambda: gs.torus_graph(37, 73, "pm1"),
    lambda: gs.er_graph(1601, 0.004, 74, "pm1"),
    lambda: gs.rgg_graph(700, 40.0, 75, "unit"),
]


@pytest.mark.parametrize("tune", [None, dict(block=64, lanes_per_node=1, grid=3),
                                  dict(block=256, lanes_per_node=8), dict(block=1024, lanes_per_node=64, grid=1000),
                                  dict(block=256, batch_members=-1), dict(block=256, batch_members=4, grid=24),
                                  dict(block=512, batch_members=16, lanes_per_node=2)])
@pytest.mark.parametrize("mode", [0, 1])
def test_mixed_batch_matches_single_runs(gdi, oracle_lib, tune, mode):
    graphs = [f() for f in MIXED]
    replicas = [[0], [0, 5], [3], [0], list(range(6))]
    T = gs.geometric_temps(2.5, 0.05, 60)
    print(f"[case] mixed batch tune={tune} mode={mode}", flush=True)
    anns, items, cases = make_items(gdi, graphs, replicas)
    out = gdi.anneal_batch(items, T, 17, mode=mode, tune=tune)
    refs = oracle_runs(oracle_lib, cases, T, 17, mode=mode)
    for i, ref in enumerate(refs):
        assert np.array_equal(out["spins"][i], ref["spins"]), i
        assert (out["M"][i], out["cut"][i]) == (ref["M"], ref["cut"]), i
    for a in anns:
        a.close()


def test_batch_equals_plain_anneal(gdi):
    """The batch result of an instance equals gdi_anneal of the same instance."""
    g = gs.er_graph(2000, 0.01, 76)
    T = gs.geometric_temps(2.0, 0.05, 100)
    with gdi.Annealer(g) as a:
        out = gdi.anneal_batch([(a.h, g.n, r) for r in range(4)], T, 9)
        for r in range(4):
            single = a.anneal(T, 9, replica=r)
            assert np.array_equal(single["spins"], out["spins"][r])
            assert (single["M"], single["cut"]) == (out["M"][r], out["cut"][r])


def test_full_batched_workload(gdi, oracle_lib):
    """64 uneven graphs (n 800-20000, mean degree 4-48) plus 256 replicas of one n=2000 graph,
    1000 sweeps, one launch; every instance against the oracle."""
    graphs = gs.batch_mix()
    g2000 = gs.er_graph(2000, 0.01, 103, "unit")
    T = gs.geometric_temps(2.0, 0.05, 1000)
    anns, items, cases = make_items(gdi, graphs + [g2000], [[0]] * len(graphs) + [list(range(256))])
    print(f"[case] full batch: {len(items)} instances, sum n = {sum(i[1] for i in items)}", flush=True)
    out = gdi.anneal_batch(items, T, 1)
    print(f"batch kernel {out['kernel_ms']:.1f} ms", flush=True)
    refs = oracle_runs(oracle_lib, cases, T, 1)
    bad = [i for i, ref in enumerate(refs)
           if not (np.array_equal(out["spins"][i], ref["spins"]) and out["M"][i] == ref["M"]
                   and out["cut"][i] == ref["cut"])]
    assert not bad, bad[:10]
    for a in anns:
        a.close()


def test_autotuner_choice_is_valid_and_result_invariant(gdi, oracle_lib):
    graphs = [f() for f in MIXED[:3]]
    T = gs.geometric_temps(2.0, 0.05, 40)
    anns, items, cases = make_items(gdi, graphs, [[0, 1]] * 3)
    best, ms = gdi.autotune_batch(items, T, 5, probe_sweeps=5)
    assert best["block"] in (128, 256, 512, 1024) and ms > 0
    tuned = gdi.anneal_batch(items, T, 5, tune=best)
    auto = gdi.anneal_batch(items, T, 5)
    refs = oracle_runs(oracle_lib, cases, T, 5)
    for i, ref in enumerate(refs):
        assert np.array_equal(tuned["spins"][i], ref["spins"])
        assert np.array_equal(auto["spins"][i], ref["spins"])
    for a in anns:
        a.close()


def test_batch_device_outputs(gdi, oracle_lib):
    import torch

    g = gs.rgg_graph(5000, 8.0, 77)
    T = gs.geometric_temps(3.0, 0.05, 50)
    outs = [torch.zeros(g.n, dtype=torch.int8, device="cuda:0") for _ in range(3)]
    with gdi.Annealer(g) as a:
        res = gdi.anneal_batch([(a.h, g.n, r) for r in range(3)], T, 4,
                               device_outputs=[o.data_ptr() for o in outs])
    for r in range(3):
        ref = oracle_lib.anneal(g, T, 4, replica=r)
        assert np.array_equal(outs[r].cpu().numpy(), ref["spins"])
        assert res["M"][r] == ref["M"]


def test_batch_rejects_bad_input(gdi):
    g = gs.er_graph(300, 0.05, 78)
    with gdi.Annealer(g) as a:
        with pytest.raises(gdi.GdiError) as e:
            gdi.anneal_batch([], np.ones(3), 1)
        assert e.value.code == gdi.EINVAL
        with pytest.raises(gdi.GdiError) as e:
            gdi.anneal_batch([(None, g.n, 0)], np.ones(3), 1)
        assert e.value.code == gdi.EINVAL
        with pytest.raises(gdi.GdiError) as e:
            gdi.anneal_batch([(a.h, g.n, 0)], np.array([1.0, -1.0]), 1)
        assert e.value.code == gdi.EINVAL
