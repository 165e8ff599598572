"""CPU-side checks of the C ABI: symbols, host logic, validation and error codes (no GPU)."""
import os
import re
import subprocess
import sys

import numpy as np
import pytest

import gdi_synth as gs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gdi():
    import paper_1908_00210_amd as gdi
    from paper_1908_00210_amd import build

    if build.is_stale():
        build.build()
    gdi.lib()
    return gdi


def declared_functions():
    with open(os.path.join(ROOT, "include", "gdi.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(gdi_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol(gdi):
    names = declared_functions()
    assert len(names) >= 15
    out = subprocess.run(["nm", "-D", "--defined-only", gdi.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = set(re.findall(r"\sT\s(gdi_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert set(names) == set(gdi.SIGNATURES)  # the binding covers exactly the header


def test_host_tables_agree_with_oracle(gdi, oracle_lib):
    """Library and oracle build the same colouring, thresholds and Philox words independently."""
    for g in (gs.er_graph(300, 0.05, 1), gs.rgg_graph(5000, 8.0, 2), gs.torus_graph(30, 3)):
        c1, C1 = gdi.colour_csr(g.row_ptr, g.col, g.n)
        c2, C2 = oracle_lib.colour(g)
        assert C1 == C2 and np.array_equal(c1, c2)
    T = np.concatenate([gs.geometric_temps(3.0, 0.05, 2000), [1e300, 1e-3, 17.0]])
    assert np.array_equal(gdi.threshold_table(T, 120), oracle_lib.thresholds(T, 120))
    rng = np.random.default_rng(3)
    for _ in range(200):
        seed = int(rng.integers(0, 2**63))
        ctr = rng.integers(0, 2**32, size=4, dtype=np.uint64).astype(np.uint32)
        assert np.array_equal(gdi.philox4x32_10(seed, ctr), oracle_lib.philox(seed, [ctr])[0])


def _err(gdi, fn, *a):
    with pytest.raises(gdi.GdiError) as e:
        fn(*a)
    return e.value.code


def test_create_rejects_malformed_csr(gdi):
    g = gs.er_graph(50, 0.2, 4, "pm1")
    rp, col, w = g.row_ptr.copy(), g.col.copy(), g.w.copy()
    E = gdi.EINVAL
    assert _err(gdi, gdi.create, rp, col, w, 1) == E                       # n < 2
    bad = rp.copy(); bad[0] = 1
    assert _err(gdi, gdi.create, bad, col, w, g.n) == E                     # row_ptr[0] != 0
    bad = rp.copy(); bad[5] = bad[6] + 1
    assert _err(gdi, gdi.create, bad, col, w, g.n) == E                     # decreasing
    bad = col.copy(); bad[3] = g.n
    assert _err(gdi, gdi.create, rp, bad, w, g.n) == E                      # out of range
    bad = col.copy(); bad[rp[7]] = 7
    assert _err(gdi, gdi.create, rp, bad, w, g.n) == E                      # self-loop
    bad = col.copy(); k = rp[9]; bad[k + 1] = bad[k]
    assert _err(gdi, gdi.create, rp, bad, w, g.n) == E                      # duplicate
    bad = w.copy(); bad[rp[11]] += 1
    assert _err(gdi, gdi.create, rp, col, bad, g.n) == E                    # asymmetric weight
    # a directed-only edge: drop the mirror of one entry
    i = 12; j = col[rp[i]]
    keep = np.ones(col.size, bool)
    mirror = rp[j] + np.searchsorted(col[rp[j]:rp[j + 1]], i)
    keep[mirror] = False
    rp2 = rp.copy(); rp2[j + 1:] -= 1
    assert _err(gdi, gdi.create, rp2, col[keep], w[keep], g.n) == E
    big = np.full_like(w, 2**29)
    assert _err(gdi, gdi.create, rp, col, big, g.n) == gdi.ERANGE           # sum |w| > 2^30


def test_create_without_gpu_reports_device_error(gdi):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    g = gs.er_graph(40, 0.2, 5)
    assert _err(gdi, gdi.create, g.row_ptr, g.col, g.w, g.n) == gdi.EDEVICE
    assert "device" in gdi.lib().gdi_last_error().decode().lower()


def test_null_handle_is_a_state_error(gdi):
    assert _err(gdi, gdi.last_result, None) == gdi.ESTATE
    assert _err(gdi, gdi.cut, None, np.ones(4, np.int8)) == gdi.ESTATE
    gdi.destroy(None)  # no-op


def test_binding_fails_loudly_without_library(tmp_path):
    code = ("import paper_1908_00210_amd as g\n"
            "g.LIB_PATH = '/nonexistent/libgdi.so'\n"
            "try:\n    g.lib()\nexcept ImportError as e:\n    print('raised', e)\n")
    out = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True)
    assert "raised" in out.stdout


def test_bench_refuses_more_than_one_gpu():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True)
    assert out.returncode != 0 and "one GPU" in out.stderr


def test_no_product_code_touches_the_oracle():
    """The HIP path never imports or links the oracle (and the oracle never the HIP path)."""
    pkg = os.path.join(ROOT, "paper_1908_00210_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".cpp", ".h")):
                with open(os.path.join(dirpath, fn)) as f:
                    assert "oracle" not in f.read().lower(), fn
    for fn in os.listdir(os.path.join(ROOT, "oracle")):
        if fn.endswith((".py", ".c")):
            with open(os.path.join(ROOT, "oracle", fn)) as f:
                assert "paper_1908_00210_amd" not in f.read(), fn
