"""The C ABI library loads and exports every entry point include/lsort.h
declares; argument errors are reported without touching a GPU."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lsort.h")


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_entry_points():
    names = declared()
    for n in ("ls_sort", "ls_sort_segmented", "ls_workspace_bytes", "ls_set_workspace", "ls_get_stats",
              "ls_last_error", "ls_rmi_fit", "ls_rmi_buckets", "ls_partition_rmi", "ls_splitters"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2307_08637_amd import lsort
    lib = lsort.lib()
    for name in declared():
        assert hasattr(lib, name), name
    assert lsort.version().startswith("lsort")


def test_struct_sizes_match_header(tmp_path):
    """The binding's ctypes structs have the C compiler's layout of the header."""
    import shutil
    import subprocess
    from paper_2307_08637_amd import lsort
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    prog = tmp_path / "sz.c"
    prog.write_text('#include "lsort.h"\n#include <stdio.h>\n#include <stddef.h>\n'
                    'int main(void){printf("%zu %zu %zu %zu\\n", sizeof(ls_options), sizeof(ls_stats),'
                    ' offsetof(ls_options, seed), offsetof(ls_stats, level));return 0;}\n')
    exe = tmp_path / "sz"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)], check=True)
    a, b, c, d = map(int, subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split())
    assert C.sizeof(lsort.Options) == a
    assert C.sizeof(lsort.Stats) == b
    assert lsort.Options.seed.offset == c
    assert lsort.Stats.level.offset == d


def test_argument_errors_without_gpu():
    from paper_2307_08637_amd import lsort
    lib = lsort.lib()
    o = lsort.make_options()
    # bad dtype, null keys with n > 0, misaligned keys: rejected before any HIP call
    assert lib.ls_sort(None, 10, 0, None, C.byref(o), None) == -1
    assert b"NULL" in lib.ls_last_error()
    assert lib.ls_sort(C.c_void_p(8), 10, 7, None, C.byref(o), None) == -1
    assert lib.ls_sort(C.c_void_p(12), 10, 0, None, C.byref(o), None) == -1
    bad = lsort.make_options(buckets=5000)
    assert lib.ls_sort(C.c_void_p(64), 10, 0, None, C.byref(bad), None) == -1
    assert b"buckets" in lib.ls_last_error()
    wrong = lsort.make_options()
    wrong.struct_size = 4
    assert lib.ls_sort(C.c_void_p(64), 10, 0, None, C.byref(wrong), None) == -1
    # n = 0 and n = 1 are no-ops
    assert lib.ls_sort(None, 0, 0, None, None, None) == 0
    assert lib.ls_sort(C.c_void_p(64), 1, 1, None, None, None) == 0


def test_stream_argument_errors_without_gpu():
    from paper_2307_08637_amd import lsort
    lib = lsort.lib()
    assert lib.ls_stream_copy(None, None, 5, None) == -1
    assert b"NULL" in lib.ls_last_error()
    assert lib.ls_stream_copy(C.c_void_p(64), C.c_void_p(68), 5, None) == -1
    assert b"aligned" in lib.ls_last_error()
    assert lib.ls_stream_read(C.c_void_p(64), 5, None, None) == -1
    assert lib.ls_stream_read(C.c_void_p(12), 5, C.c_void_p(64), None) == -1
    assert b"aligned" in lib.ls_last_error()
    assert lib.ls_stream_copy(None, None, 0, None) == 0


def test_workspace_bytes_host_only():
    from paper_2307_08637_amd import lsort
    small = lsort.workspace_bytes(10**6)
    big = lsort.workspace_bytes(10**8)
    assert 0 < small < big
    assert lsort.workspace_bytes(10**6, payload=True) > small


TABLE = """{
  "format": "lsort-tuning-1",
  "device": "%s",
  "cus": %d,
  "classes": [
    {"log10_avg_size": 3, "buckets": 256, "cutoff": 256, "tree_buckets": 128, "ms": 1.0, "default_ms": 1.2},
    {"log10_avg_size": 6, "buckets": 512, "cutoff": 512, "tree_buckets": 256, "ms": 2.0, "default_ms": 2.1},
    {"log10_avg_size": 8, "buckets": 1000, "cutoff": 256, "tree_buckets": 256, "tile": 131072, "ms": 4.0,
     "default_ms": 4.5}
  ]
}
"""


def test_tuning_table_lookup(tmp_path):
    """Loading a table changes exactly the tuned fields, by size class (the
    nearest class present), and unloading restores the defaults.  No GPU is
    touched: without a device the table's device key is not compared."""
    import torch
    from paper_2307_08637_amd import lsort
    if torch.cuda.is_available():
        pytest.skip("the device-key check needs a table made on this device; covered by the GPU tests")
    path = tmp_path / "t.json"
    path.write_text(TABLE % ("gfx950", 256))
    defaults = lsort.tuned_options(10**6, 1)
    assert defaults["buckets"] == 1000 and defaults["cutoff"] == 1024 and defaults["tree_buckets"] == 256
    assert lsort.tuned_options(10**6, 100)["cutoff"] == 512  # the segmented form's default
    lsort.load_tuning(str(path))
    try:
        assert lsort.tuned_options(10**6, 1) == {"buckets": 512, "cutoff": 512, "tree_buckets": 256, "leaves": 1000,
                                                 "tile": 32768}  # no tile in the entry: the default
        assert lsort.tuned_options(10**8, 1)["tile"] == 131072
        assert lsort.tuned_options(2 * 10**7, 20_000)["buckets"] == 256          # class 3
        assert lsort.tuned_options(10**8, 1)["cutoff"] == 256                    # class 8
        assert lsort.tuned_options(10**4, 1)["buckets"] == 256                   # class 4 -> nearest 3
        assert lsort.tuned_options(3 * 10**7, 1)["buckets"] == 512               # class 7: tie, smaller class (6)
    finally:
        lsort.load_tuning(None)
    assert lsort.tuned_options(10**6, 1) == defaults


@pytest.mark.parametrize("text", ["{}", '{"format": "other"}',
                                  TABLE.replace('"buckets": 512', '"buckets": 5000') % ("gfx950", 256),
                                  TABLE.replace('"tree_buckets": 128', '"tree_buckets": 100') % ("gfx950", 256),
                                  TABLE.replace('"tile": 131072', '"tile": 100000') % ("gfx950", 256)])
def test_tuning_table_rejects_bad_files(tmp_path, text):
    import torch
    from paper_2307_08637_amd import lsort
    if torch.cuda.is_available():
        pytest.skip("CPU-only check")
    path = tmp_path / "bad.json"
    path.write_text(text)
    with pytest.raises(lsort.LsortError):
        lsort.load_tuning(str(path))
    with pytest.raises(lsort.LsortError):
        lsort.load_tuning(str(tmp_path / "missing.json"))
