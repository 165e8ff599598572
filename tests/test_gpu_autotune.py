"""The single-graph autotuner (gdi_autotune) and its cache, on the GPU.

Whatever launch the tuner installs, the anneal's result is the oracle's (launch choices
never change a trajectory); a cached choice is installed again without timing, also
after the cache went through a JSON file.
"""
import ctypes

import numpy as np
import pytest

import gdi_synth as gs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gdi():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_00210_amd as gdi

    gdi.lib()
    return gdi


@pytest.mark.parametrize("n,deg,seed", [(3001, 10.0, 13), (40000, 8.0, 21)])
def test_autotuned_launch_keeps_the_trajectory(gdi, oracle_lib, tmp_path, n, deg, seed):
    g = gs.rgg_graph(n, deg, seed, "pm1")
    T = gs.geometric_temps(3.0, 0.05, 40)
    print(f"[case] autotune n={n} deg={deg} seed={seed}", flush=True)
    gdi.tune_cache_clear()
    with gdi.Annealer(g) as a:
        best, ms = a.autotune(T, 7, probe_sweeps=10)
        print(f"autotune n={n}: {best} {ms:.3f} ms per 10 sweeps", flush=True)
        assert ms > 0 and best.get("scope") in (gdi.SCOPE_WORKGROUP, gdi.SCOPE_GRID)
        r = a.anneal(T, 7)
        if n > 65536:
            assert best["scope"] == gdi.SCOPE_GRID
        # the cache, through a file, gives the same choice back without timing
        path = str(tmp_path / "tune.json")
        gdi.tune_cache_save(path)
        gdi.tune_cache_clear()
        gdi.tune_cache_load(path)
        a.tune(reset=True)
        best2, ms2 = a.autotune(T, 7, probe_sweeps=10, use_cache=True)
        assert best2 == best and ms2 == ms
        r2 = a.anneal(T, 7)
    ref = oracle_lib.anneal(g, T, 7)
    assert np.array_equal(r["spins"], ref["spins"]) and np.array_equal(r2["spins"], ref["spins"])
    assert r["cut"] == ref["cut"] and r["M"] == ref["M"]
    gdi.tune_cache_clear()


def test_autotune_rejects_racy_schedules(gdi):
    g = gs.rgg_graph(2000, 8.0, 3, "pm1")
    with gdi.Annealer(g) as a:
        s, T = gdi._schedule(np.ones(4), 1, 1, 0, gdi.BAL_GATED, 0, None, None, None, flags=gdi.FLAG_RACY)
        best = gdi.Tuning()
        rc = gdi.lib().gdi_autotune(a.h, ctypes.byref(s), ctypes.c_uint64(1), 2, 0, ctypes.byref(best), None)
        assert rc == gdi.EINVAL
        # the handle's tuning is untouched: the automatic launch still runs
        r = a.anneal(np.ones(3), 1)
        assert r["result"]["scope"] == gdi.SCOPE_WORKGROUP
