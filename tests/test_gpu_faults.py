"""Failure paths on the GPU: device allocations that fail (GDI_FAULT=alloc makes every
device allocation of the library fail as if the device were out of memory).

Each failing call must return GDI_ENOMEM with a message and leave the library
usable: once the variable is cleared, the same handle anneals bit for bit like the
oracle. The allocation-free cut must still work while allocations fail.
"""
import os

import numpy as np
import pytest

import gdi_synth as gs

pytestmark = pytest.mark.gpu


@pytest.fixture()
def alloc_fault():
    os.environ["GDI_FAULT"] = "alloc"
    try:
        yield
    finally:
        os.environ.pop("GDI_FAULT", None)


def test_failed_allocations_report_enomem_and_recover(oracle_lib, alloc_fault):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_00210_amd as gdi

    g = gs.rgg_graph(3000, 8.0, 71, "pm1")
    T = gs.geometric_temps(2.5, 0.05, 40)
    print("[case] gdi_create under GDI_FAULT=alloc", flush=True)
    with pytest.raises(gdi.GdiError) as e:
        gdi.Annealer(g)
    assert e.value.code == gdi.ENOMEM and "hipMalloc" in str(e.value)
    os.environ.pop("GDI_FAULT")
    a = gdi.Annealer(g)
    try:
        spins = np.where(np.random.default_rng(3).random(g.n) < 0.5, 1, -1).astype(np.int8)
        d_spins = torch.from_numpy(spins).to("cuda:0")
        d_out = torch.zeros(3, dtype=torch.int64, device="cuda:0")
        a.set_stream(torch.cuda.current_stream().cuda_stream)
        a.anneal(T[:2], 1)  # threshold table and launch state of a short schedule
        os.environ["GDI_FAULT"] = "alloc"
        print("[case] calls that allocate, under GDI_FAULT=alloc", flush=True)
        with pytest.raises(gdi.GdiError) as e:
            a.cut(spins)  # allocates its scratch per call
        assert e.value.code == gdi.ENOMEM
        with pytest.raises(gdi.GdiError) as e:
            a.anneal(T, 1)  # a longer schedule needs a larger threshold table
        assert e.value.code == gdi.ENOMEM
        # the allocation-free entry point allocates nothing
        a.cut_dev_noalloc(d_spins.data_ptr(), d_out.data_ptr())
        torch.cuda.current_stream().synchronize()
        assert tuple(int(x) for x in d_out.cpu().numpy()) == tuple(oracle_lib.cut(g, spins))
        os.environ.pop("GDI_FAULT")
        print("[case] recovery", flush=True)
        # the short schedule's table was released by the failed reallocation: it must be
        # built again, not taken from a stale cache entry
        ref2 = oracle_lib.anneal(g, T[:2], 1)
        r2 = a.anneal(T[:2], 1)
        assert np.array_equal(r2["spins"], ref2["spins"]) and (r2["M"], r2["cut"]) == (ref2["M"], ref2["cut"])
        ref = oracle_lib.anneal(g, T, 1)
        r = a.anneal(T, 1)
        assert np.array_equal(r["spins"], ref["spins"]) and (r["M"], r["cut"]) == (ref["M"], ref["cut"])
        assert a.cut(spins) == tuple(oracle_lib.cut(g, spins))
    finally:
        a.close()
