"""The C-ABI library loads and exports every entry point its headers declare (no GPU needed),
and the binding fails loudly when the library is missing."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2606_22332_amd", "libtg_readout.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[\w\s\*]+?\b(tg_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("tg_readout_create", "tg_readout_step", "tg_readout_rollout", "tg_readout_destroy",
              "tg_readout_reset", "tg_readout_last_error", "tg_status_string"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_status_strings_and_null_handling():
    lib = ctypes.CDLL(LIB)
    lib.tg_status_string.restype = ctypes.c_char_p
    assert lib.tg_status_string(0) == b"ok"
    assert lib.tg_status_string(1) == b"invalid argument"
    lib.tg_readout_destroy.argtypes = [ctypes.c_void_p]
    assert lib.tg_readout_destroy(None) == 0
    lib.tg_readout_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    assert lib.tg_readout_create(None, None) == 1          # rejected on the host, nothing launched
    lib.tg_readout_step.argtypes = [ctypes.c_void_p] * 4
    assert lib.tg_readout_step(None, None, None, None) == 1
    lib.tg_readout_poll_errors.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
    flags = ctypes.c_uint32(7)
    assert lib.tg_readout_poll_errors(None, ctypes.byref(flags)) == 1 and flags.value == 7


def test_binding_raises_without_library(tmp_path, monkeypatch):
    from paper_2606_22332_amd import binding
    monkeypatch.setattr(binding, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(binding, "_lib", None)
    with pytest.raises(binding.TgError):
        binding.load()


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_unstable_thermal_configuration_is_rejected_at_create():
    """The positivity bound of the explicit thermal step is checked before any device work."""
    from paper_2606_22332_amd import binding as B
    from paper_2606_22332_amd import synth
    import ctypes as C
    sc = synth.make_scene("c5", num_envs=2, num_steps=1)
    sc.thermal.dt = 2.0                     # r = alpha dt / dx^2 = 0.2 > 1/6
    lib = B.load()
    keep = []
    cfg = B.make_config(sc, B.OUT_ALL, keep)
    h = C.c_void_p()
    rc = lib.tg_readout_create(C.byref(cfg), C.byref(h))
    assert rc == 5 and not h.value             # TG_ERR_UNSTABLE
    assert b"stable" in lib.tg_readout_last_error(None)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
@pytest.mark.parametrize("field,value,status", [
    ("num_envs", 0, 1),                     # sizes must be positive
    ("num_taxels", 0, 1),
    ("num_envs", 1 << 20, 4),               # E * T * 4 bytes past 2^32: shard the envs
    ("abi_version", 99, 1),
])
def test_create_rejects_bad_sizes_on_the_host(field, value, status):
    """Size and version errors are found on the host before any device call (here, where no
    GPU exists, a call that got past them would fail differently)."""
    from paper_2606_22332_amd import binding as B
    from paper_2606_22332_amd import synth
    import ctypes as C
    sc = synth.make_scene("c3", num_envs=4, num_steps=1)
    lib = B.load()
    keep = []
    cfg = B.make_config(sc, B.OUT_ALL, keep)
    setattr(cfg, field, value)
    h = C.c_void_p()
    assert lib.tg_readout_create(C.byref(cfg), C.byref(h)) == status and not h.value
