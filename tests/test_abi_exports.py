"""CPU-side checks of the boundary: the built library loads and exports every
entry point include/pdit.h declares (no compute calls, no GPU needed)."""
import ctypes
import os
import re

import pytest

from conftest import ROOT

HEADER = os.path.join(ROOT, "include", "pdit.h")
LIB = os.path.join(ROOT, "paper_2605_24408_amd", "libpdit.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pdit_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("pdit_create", "pdit_destroy", "pdit_run_sweeps", "pdit_energy",
                     "pdit_best", "pdit_run_sweeps_batch", "pdit_h_recompute"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpdit.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpdit.so not built")
def test_binding_declares_every_export():
    from paper_2605_24408_amd import pdit
    assert sorted(pdit.EXPORTS) == declared_functions()


def test_library_sources_do_not_touch_the_oracle():
    csrc = os.path.join(ROOT, "paper_2605_24408_amd")
    for dirpath, _, files in os.walk(csrc):
        for f in files:
            if f.endswith((".hip", ".h", ".py", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower() or f == "workloads.py", f


def header_struct_fields(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r";", text).group(1)
    return re.findall(r"\b([a-z_][a-z0-9_]*)\s*;", body)


def test_binding_matches_header_options_and_codes():
    from paper_2605_24408_amd import pdit
    assert [f[0] for f in pdit._Opts._fields_] == header_struct_fields("pdit_opts")
    text = open(HEADER).read()
    codes = {int(v): k for k, v in re.findall(r"#define (PDIT_(?:OK|E[A-Z]+))\s+\(?(-?\d+)\)?", text)}
    assert codes == pdit.STATUS


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpdit.so not built")
def test_default_options_on_the_host():
    """pdit_default_opts only fills the struct (no device call): the ctypes
    layout reads back the documented defaults."""
    from paper_2605_24408_amd import pdit
    lib = ctypes.CDLL(LIB)
    o = pdit._Opts()
    ctypes.memset(ctypes.byref(o), 0x5A, ctypes.sizeof(o))
    lib.pdit_default_opts(ctypes.byref(o))
    assert (o.device, o.stream, o.recompute, o.sweep, o.blocks_per_cu, o.seq_threshold,
            o.paranoid) == (0, None, 0, 0, 0, -1, 0)
