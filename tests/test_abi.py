"""CPU checks of the C ABI library: it loads (without a GPU) and exports
every function include/gm.h declares.  No compute calls."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2602_13198_amd", "_lib", "libgm.so")


def declared():
    src = open(os.path.join(ROOT, "include", "gm.h")).read()
    return sorted(set(re.findall(r"^\s*(?:gm_status|const char \*)\s*(gm_\w+)\s*\(", src, re.M)))


def test_header_declarations_are_complete():
    from paper_2602_13198_amd import gm as binding   # noqa: F401  (torch imported first)
    names = declared()
    assert "gm_track_scatter" in names and len(names) >= 12
    assert sorted(binding.EXPORTS) == names


def test_library_exports_every_symbol():
    import torch  # noqa: F401  (share torch's HIP runtime)
    if not os.path.exists(LIB):
        import __graft_entry__
        __graft_entry__.build()
    L = ctypes.CDLL(LIB)
    for name in declared():
        assert hasattr(L, name), name


def test_structs_match_header_layout(tmp_path):
    """ctypes mirrors have the sizes and field offsets gcc gives the header."""
    import subprocess
    from paper_2602_13198_amd import gm as b
    prog = tmp_path / "sz.c"
    prog.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "%s/include/gm.h"\n'
                    'int main(){printf("%%zu %%zu %%zu %%zu %%zu %%zu %%zu\\n", sizeof(gm_grid),'
                    'sizeof(gm_zones), sizeof(gm_emit_params), sizeof(gm_track_params),'
                    'sizeof(gm_trace_rec), offsetof(gm_track_params, max_steps),'
                    'offsetof(gm_track_params, precision));}' % ROOT)
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-o", str(exe), str(prog)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True,
                                          check=True).stdout.split()]
    want = [ctypes.sizeof(b.GmGrid), ctypes.sizeof(b.GmZones), ctypes.sizeof(b.GmEmitParams),
            ctypes.sizeof(b.GmTrackParams), b.TRACE_BYTES,
            b.GmTrackParams.max_steps.offset, b.GmTrackParams.precision.offset]
    assert got == want
