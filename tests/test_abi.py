"""The C-ABI library loads and exports every entry point its header declares,
and the binding's struct layouts match the header's (checked by compiling a
tiny host program against the header).  No compute calls: no GPU here."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

import paper_1808_05458_amd as mc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(mc.HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(mc_[a-z_]+)\s*\(",
                       text, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(mc.library_path()):
        mc.build()
    return ctypes.CDLL(mc.library_path())


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["mc_mincut", "mc_mincut_batched", "mc_workspace_bytes", "mc_strerror",
                     "mc_options_default", "mc_release", "mc_timing_get", "mc_timing_reset"]:
        assert required in names


def test_every_declared_symbol_is_exported(lib):
    out = subprocess.run(["nm", "-D", "--defined-only", mc.library_path()], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r"\s[TW]\s+(\S+)$", out, flags=re.M))
    for name in declared_functions():
        assert name in exported, name
        assert hasattr(lib, name)


def test_error_strings_and_defaults(lib):
    lib.mc_strerror.restype = ctypes.c_char_p
    for code in range(-9, 1):
        assert lib.mc_strerror(code)
    o = mc.options()
    assert o.use_pr == 1 and o.eager_blacklist == 1 and o.timing == 0
    lib.mc_workspace_bytes.restype = ctypes.c_size_t
    lib.mc_workspace_bytes.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32]
    small = lib.mc_workspace_bytes(1000, 10000, 1)
    big = lib.mc_workspace_bytes(1 << 22, 1 << 27, 1)
    assert 0 < small < big


def test_struct_layouts_match_header():
    src = r"""
    #include <stdio.h>
    #include <stddef.h>
    #include "mincut.h"
    int main(void) {
      printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(mc_graph), sizeof(mc_batch),
             sizeof(mc_options), sizeof(mc_stats), sizeof(mc_timing_entry),
             offsetof(mc_stats, ms), offsetof(mc_options, timing), sizeof(mc_server_cfg),
             sizeof(mc_request), sizeof(mc_latency), offsetof(mc_server_cfg, opt),
             offsetof(mc_options, sort_tile), sizeof(mc_tune_result), offsetof(mc_tune_result, best_ms));
      return 0;
    }
    """
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        open(c, "w").write(src)
        exe = os.path.join(d, "t")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(x) for x in subprocess.check_output([exe]).split()]
    assert vals[0] == ctypes.sizeof(mc.Graph)
    assert vals[1] == ctypes.sizeof(mc.Batch)
    assert vals[2] == ctypes.sizeof(mc.Options)
    assert vals[3] == ctypes.sizeof(mc.Stats)
    assert vals[4] == ctypes.sizeof(mc.TimingEntry)
    assert vals[7] == ctypes.sizeof(mc.ServerCfg)
    assert vals[8] == ctypes.sizeof(mc.Request)
    assert vals[9] == ctypes.sizeof(mc.Latency)
    assert vals[10] == mc.ServerCfg.opt.offset
    assert vals[5] == mc.Stats.ms.offset
    assert vals[6] == mc.Options.timing.offset
    assert vals[11] == mc.Options.sort_tile.offset
    assert vals[12] == ctypes.sizeof(mc.TuneResult)
    assert vals[13] == mc.TuneResult.best_ms.offset


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    monkeypatch.setattr(mc, "_lib", None)
    monkeypatch.setattr(mc, "_LIB", str(tmp_path / "absent.so"))
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        mc._load()
