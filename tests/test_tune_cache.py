"""The autotuners' persisted cache (gdi_tune_cache_* and GDI_TUNE_CACHE), on the CPU.

The JSON reader and writer are checked under the address and undefined-behaviour
sanitizers (tests/tunecache_check.cpp); the C ABI's load, save, clear and size, and the
environment variable, through the built library. No GPU: the cache itself makes no HIP
call (the tuners that fill it are covered by the GPU tests).
"""
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def gdi():
    import paper_1908_00210_amd as gdi
    from paper_1908_00210_amd import build

    if build.is_stale():
        build.build()
    gdi.lib()
    return gdi


ENTRY = {"scope": 2, "block": 1024, "grid": 128, "lanes_per_node": 1, "tail_max": 0, "leaders": 0,
         "general_weights": 0, "csr_lds": 0, "batch_members": 0, "ms": 3.25}


def write(path, obj):
    with open(path, "w") as f:
        f.write(obj if isinstance(obj, str) else json.dumps(obj))


def test_parser_under_sanitizers(tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ is not available")
    exe = str(tmp_path / "tunecache_check")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-Wall", "-Wextra", "-Werror", "-o", exe,
           os.path.join(ROOT, "tests", "tunecache_check.cpp"),
           os.path.join(ROOT, "paper_1908_00210_amd", "csrc", "gdi_tunecache.cpp")]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stdout + b.stderr
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1"))
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
    assert int(r.stdout.split()[1]) > 20000


def test_load_save_round_trip(gdi, tmp_path):
    gdi.tune_cache_clear()
    assert gdi.tune_cache_size() == 0
    src = tmp_path / "in.json"
    entries = {"gfx950/256cu|graph|n=1000|nnz=6000|C=7|maxdeg=12|w=pm1": ENTRY,
               "gfx950/256cu|batch|inst=4|n=10|nnz=20|maxnpad=64|maxC=3": dict(ENTRY, scope=0, batch_members=8,
                                                                                   ms=0.5)}
    write(src, {"format": "gdi-tune-1", "entries": entries})
    gdi.tune_cache_load(str(src))
    assert gdi.tune_cache_size() == 2
    out = tmp_path / "out.json"
    gdi.tune_cache_save(str(out))
    back = json.loads(out.read_text())
    assert back["format"] == "gdi-tune-1" and back["entries"] == entries
    # loading again replaces equal keys and adds new ones
    write(src, {"format": "gdi-tune-1", "entries": {"other": ENTRY}})
    gdi.tune_cache_load(str(src))
    assert gdi.tune_cache_size() == 3
    gdi.tune_cache_clear()
    assert gdi.tune_cache_size() == 0


@pytest.mark.parametrize("text", [
    "", "not json", "{}", '{"format": "gdi-tune-2", "entries": {}}',
    '{"format": "gdi-tune-1", "entries": {"k": {"block": "256"}}}',
    '{"format": "gdi-tune-1", "entries": {"k": {"block": 256}}',
])
def test_malformed_files_are_rejected_whole(gdi, tmp_path, text):
    gdi.tune_cache_clear()
    ok = tmp_path / "ok.json"
    write(ok, {"format": "gdi-tune-1", "entries": {"a": ENTRY}})
    gdi.tune_cache_load(str(ok))
    bad = tmp_path / "bad.json"
    write(bad, text)
    with pytest.raises(gdi.GdiError) as e:
        gdi.tune_cache_load(str(bad))
    assert e.value.code == gdi.EINVAL
    assert gdi.tune_cache_size() == 1
    with pytest.raises(gdi.GdiError):
        gdi.tune_cache_load(str(tmp_path / "missing.json"))
    with pytest.raises(gdi.GdiError):
        gdi.tune_cache_save(str(tmp_path / "no_such_dir" / "x.json"))
    gdi.tune_cache_clear()


def test_environment_variable_names_the_file(gdi, tmp_path):
    """A fresh process reads GDI_TUNE_CACHE at its first lookup; a malformed file there is
    ignored rather than an error."""
    path = tmp_path / "env.json"
    write(path, {"format": "gdi-tune-1", "entries": {"a": ENTRY, "b": ENTRY}})
    code = "import paper_1908_00210_amd as g; print(g.tune_cache_size())"
    env = dict(os.environ, GDI_TUNE_CACHE=str(path), PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120, cwd=ROOT)
    assert r.returncode == 0 and r.stdout.strip() == "2", r.stdout + r.stderr
    write(path, "{broken")
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env, timeout=120, cwd=ROOT)
    assert r.returncode == 0 and r.stdout.strip() == "0", r.stdout + r.stderr
