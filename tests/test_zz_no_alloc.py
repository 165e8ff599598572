"""The allocation-free cut (gdi_cut_dev_noalloc) against gdi_cut_dev, through the C ABI.

Two calls in a row on one GPU, the second on a smaller graph than the first, so
the second runs on a scratch array that still holds the first call's values; each
result must equal gdi_cut_dev's on the same spins (and the oracle's count), bit for
bit. The results arrive in a device buffer, stream-ordered on the handle's stream.
"""
import numpy as np
import pytest

import gdi_synth as gs

pytestmark = pytest.mark.gpu


def test_noalloc_cut_matches_the_allocating_entry_point(oracle_lib):
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1908_00210_amd as gdi

    rng = np.random.default_rng(5)
    for name, g in (("rgg300k_unit", gs.rgg_graph(300_000, 8.0, 61, "unit")),
                    ("er1500_pm1", gs.er_graph(1500, 0.01, 62, "pm1"))):
        print(f"[case] noalloc cut {name} n={g.n}", flush=True)
        spins = np.where(rng.random(g.n) < 0.5, 1, -1).astype(np.int8)
        d_spins = torch.from_numpy(spins).to("cuda:0")
        d_out = torch.full((3,), -7, dtype=torch.int64, device="cuda:0")
        with gdi.Annealer(g) as a:
            a.set_stream(torch.cuda.current_stream().cuda_stream)
            a.cut_dev_noalloc(d_spins.data_ptr(), d_out.data_ptr())
            torch.cuda.current_stream().synchronize()
            got = tuple(int(x) for x in d_out.cpu().numpy())
            want = a.cut_dev(d_spins.data_ptr())
        print(f"{name}: noalloc {got}, allocating {want}", flush=True)
        assert got == tuple(want)
        assert got == tuple(oracle_lib.cut(g, spins))
