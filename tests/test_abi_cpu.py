"""Host-side checks of the C-ABI library: it loads, exports every function
include/mpmi.h declares, and the binding's structs match the header's layout.
No compute call is made (no GPU here)."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpmi.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:[\w\s\*]+?)\b(\w+)\s*\(", text, flags=re.M)
    return sorted({n for n in names if n not in ("if", "defined")})


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("koopman_fit", "rollout_batch", "safe_mask", "select_min_intervention", "mpmi_tick",
              "mpmi_model_pack", "mpmi_create", "mpmi_destroy"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_1906_02318_amd import mpmi
    lib = mpmi.library()
    out = subprocess.run(["nm", "-D", "--defined-only", mpmi.LIB_PATH], capture_output=True, text=True).stdout
    exported = {l.split()[-1] for l in out.splitlines() if " T " in l}
    for n in declared_functions():
        assert n in exported, f"{n} declared in mpmi.h but not exported"
        assert hasattr(lib, n)
    assert lib.mpmi_abi_version() == mpmi.ABI_VERSION
    assert lib.mpmi_model_bytes() % 256 == 0


def test_struct_layouts_match_header():
    from paper_1906_02318_amd import mpmi
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "mpmi.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(mpmi_system), sizeof(mpmi_selection), sizeof(mpmi_tick_desc),
         offsetof(mpmi_system, u_hi), offsetof(mpmi_selection, first_violation), offsetof(mpmi_tick_desc, block),
         offsetof(mpmi_system, eps_track));
  return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "probe.c")
        exe = os.path.join(d, "probe")
        open(c, "w").write(src)
        subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe], check=True)
        vals = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert vals == [ctypes.sizeof(mpmi.System), ctypes.sizeof(mpmi.Selection), ctypes.sizeof(mpmi.TickDesc),
                    mpmi.System.u_hi.offset, mpmi.Selection.first_violation.offset, mpmi.TickDesc.block.offset,
                    mpmi.System.eps_track.offset]


def test_header_compiles_as_c_and_cxx():
    with tempfile.TemporaryDirectory() as d:
        for lang, comp in (("c", "gcc"), ("c++", "g++")):
            src = os.path.join(d, "h." + ("c" if lang == "c" else "cpp"))
            open(src, "w").write('#include "mpmi.h"\nint main(void){return MPMI_OK;}\n')
            subprocess.run([comp, "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"), src, "-o",
                            os.path.join(d, "h_" + comp)], check=True)


def test_missing_library_fails_loudly(monkeypatch):
    from paper_1906_02318_amd import mpmi
    monkeypatch.setattr(mpmi, "_lib", None)
    monkeypatch.setattr(mpmi, "LIB_PATH", "/nonexistent/libmpmi.so")
    with pytest.raises(RuntimeError, match="missing"):
        mpmi.library()
