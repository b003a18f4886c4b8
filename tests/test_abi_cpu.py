"""CPU-side checks of the boundary: the built library loads and exports every entry point
declared in include/*.h (no compute call: there is no GPU here)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include"))) if f.endswith(".h")]


def declared_functions():
    src = "\n".join(open(h).read() for h in HEADERS)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:ngs_status|const char\*|int32_t)\s+(ngs_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_six_entry_points():
    fns = declared_functions()
    for name in ("ngs_project", "ngs_bin_sort", "ngs_render", "ngs_info_gain", "ngs_render_backward",
                 "ngs_score_batch"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    from paper_2602_08266_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2602_08266_amd import build
        build.build()
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(binding.EXPORTS) == set(declared_functions())
    lib.ngs_version.restype = ctypes.c_int32
    assert lib.ngs_version() == 1
    lib.ngs_status_string.restype = ctypes.c_char_p
    assert lib.ngs_status_string(-5) == b"degenerate normaliser"


def test_workspace_size_is_host_only():
    from paper_2602_08266_amd import binding
    b = binding.workspace_size(0, 1000, 16, max_pairs=5000)
    assert b > 1000 * 16
    assert binding.workspace_size(2, 1000, 16, max_pairs=5000, max_slots=100) > b
    try:
        binding.workspace_size(0, 10, 65)
    except binding.NgsError as e:
        assert e.status == binding.NGS_UNSUPPORTED
    else:
        raise AssertionError("k > 64 must be unsupported")


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2602_08266_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                txt = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in txt.replace("oracle/", ""), f
