"""CPU checks of the boundary: the library loads, exports every entry point
include/cc.h declares, and rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cc.h")
LIB = os.path.join(ROOT, "paper_1607_06156_amd", "libccmi.so")


def declared():
    src = open(HEADER).read()
    return re.findall(r"^\s*(?:int|int64_t|void|const char\*)\s+(cc_\w+)\s*\(", src, re.M)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_1607_06156_amd import build
        build.build()
    lib = ctypes.CDLL(LIB)
    lib.cc_last_error.restype = ctypes.c_char_p   # every test may read the message, in any order
    return lib


def test_header_declares_the_boundary():
    names = set(declared())
    for must in ["cc_label", "cc_label_ex", "cc_label_batched", "cc_label_batched_ex", "cc_router_load",
                 "cc_last_error", "cc_version", "cc_degree", "cc_degree_histograms", "cc_powerlaw_ks", "cc_csr",
                 "cc_bfs", "cc_bfs_filter", "cc_mlp_forward", "cc_mlp_sgd_step", "cc_workspace_size",
                 "cc_release_workspace", "cc_shutdown", "cc_label64", "cc_label64_ex", "cc_label_tuples",
                 "cc_label_noalloc"]:
        assert must in names


def test_every_declared_symbol_is_exported(lib):
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert missing == []


def test_version_and_defaults(lib):
    assert lib.cc_version() == 10200
    import paper_1607_06156_amd as ccmi
    opt = ccmi.Options()
    lib.cc_default_options(ctypes.byref(opt))
    assert opt.route == 0 and opt.max_passes == 0 and abs(opt.tau - 0.05) < 1e-15 and abs(opt.theta - 8.0) < 1e-15
    assert opt.check == 0 and list(opt.reserved) == [0, 0, 0]


def test_struct_layouts_match_header(lib):
    """The Python mirrors of cc_options / cc_stats have the C sizes."""
    import paper_1607_06156_amd as ccmi
    # cc_options: 2 int32, 2 double, 2 int32, a pointer, an int64, check + 3 reserved int32
    assert ctypes.sizeof(ccmi.Options) == 8 + 16 + 8 + 8 + 8 + 16
    st = ccmi.Stats()
    assert ctypes.sizeof(st) % 8 == 0
    assert ccmi.Stats.active_edges.offset % 8 == 0


def test_struct_layouts_match_compiled_header(tmp_path):
    """Every field of the Python mirrors of cc_options, cc_stats and
    cc_batch_stats sits at the offset a C compiler gives it in include/cc.h,
    and the sizes agree."""
    import shutil
    import subprocess
    import paper_1607_06156_amd as ccmi
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    mirrors = {"cc_options": ccmi.Options, "cc_stats": ccmi.Stats, "cc_batch_stats": ccmi.BatchStats,
               "cc_tuple_stats": ccmi.TupleStats, "cc_peaks": ccmi.Peaks}
    lines = []
    for cname, py in mirrors.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    src = tmp_path / "layout.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "cc.h"\nint main(void) {\n'
                   + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(ln.split()[:2]): int(ln.split()[2]) for ln in out if ln}
    for cname, py in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, f"{cname}.{fname}"


def test_invalid_arguments_rejected_on_host(lib):
    lib.cc_label.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_void_p,
                             ctypes.c_void_p]
    lib.cc_last_error.restype = ctypes.c_char_p
    assert lib.cc_label(None, None, -1, 5, None, None) == -1
    assert b"negative" in lib.cc_last_error()
    assert lib.cc_label(None, None, 3, 5, None, None) == -1        # NULL edges with m > 0
    assert lib.cc_label(None, None, 3, 0, None, None) == -1        # edges but no vertices
    assert lib.cc_label(None, None, 0, 0, None, None) == 0         # nothing to do
    lib.cc_label_batched.argtypes = [ctypes.c_void_p] * 4 + [ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
    assert lib.cc_label_batched(None, None, None, None, -2, None, None) == -1
    assert lib.cc_label_batched(None, None, None, None, 0, None, None) == 0
    lib.cc_powerlaw_ks.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p]
    assert lib.cc_powerlaw_ks(None, None, 0, None) == -1
    hx = (ctypes.c_int64 * 4096)()
    bad_tail = (ctypes.c_int32 * 2)(5000, 4095)                  # 4095 belongs in histx, not the tail
    res = (ctypes.c_double * 5)()
    assert lib.cc_powerlaw_ks(hx, bad_tail, 2, res) == -1
    assert b"below 4096" in lib.cc_last_error()
    lib.cc_router_load.argtypes = [ctypes.c_char_p]
    assert lib.cc_router_load(b"/nonexistent/weights.txt") == -1


def test_workspace_size_and_checks(lib):
    """cc_workspace_size grows with m and n, is smaller for the forced SV
    routes (no degree pass), rejects bad arguments; a caller workspace below
    it is refused before any device work."""
    import paper_1607_06156_amd as ccmi
    L = ccmi.lib()
    sv = L.cc_workspace_size(1 << 20, 1 << 18, ccmi.ROUTE_SV)
    full = L.cc_workspace_size(1 << 20, 1 << 18, ccmi.ROUTE_AUTO)
    assert 0 < sv < full
    assert 20 * (1 << 20) <= sv <= 21 * (1 << 20) + (1 << 20)     # ~20 B per edge plus fixed tables
    assert L.cc_workspace_size(1 << 21, 1 << 18, ccmi.ROUTE_SV) > sv
    assert L.cc_workspace_size(1 << 20, 1 << 19, ccmi.ROUTE_AUTO) > full
    assert L.cc_workspace_size(1 << 20, 1 << 18, ccmi.ROUTE_SV_THETA) == sv
    assert L.cc_workspace_size(-1, 5, 0) == -1 and L.cc_workspace_size(1, 5, 9) == -1
    opt = ccmi.Options()
    L.cc_default_options(ctypes.byref(opt))
    opt.workspace = 4096                                      # never dereferenced: refused on size
    opt.workspace_bytes = 1024
    assert L.cc_label_ex(8, 8, 1000, 100, 8, None, ctypes.byref(opt), None) == -1
    assert b"workspace" in L.cc_last_error()
    opt.workspace_bytes = 0
    assert L.cc_label_ex(8, 8, 1000, 100, 8, None, ctypes.byref(opt), None) == -1
    opt.workspace = None
    opt.scratch = 7
    assert L.cc_label_ex(8, 8, 1000, 100, 8, None, ctypes.byref(opt), None) == -1


def test_check_and_failure_hook_reject_bad_arguments_on_host(lib):
    """cc_check_labels and cc_debug_fail_alloc validate on the host before
    any device work; an empty vertex set with edges reports every edge out of
    range without touching the device."""
    import paper_1607_06156_amd as ccmi
    L = ccmi.lib()
    bad = (ctypes.c_int64 * 3)(7, 7, 7)
    assert L.cc_check_labels(None, None, 0, 5, None, None, None) == -1          # NULL result
    assert L.cc_check_labels(None, None, -1, 5, None, None, bad) == -1
    assert L.cc_check_labels(None, None, 3, 5, 8, None, bad) == -1               # NULL edges
    assert L.cc_check_labels(8, 8, 3, 5, None, None, bad) == -1                  # NULL labels
    assert L.cc_check_labels(8, 8, 3, 0, None, None, bad) == 0 and list(bad) == [0, 0, 3]
    assert L.cc_check_labels(None, None, 0, 0, None, None, bad) == 0 and list(bad) == [0, 0, 0]
    assert L.cc_debug_fail_alloc(-1) == -1 and b"negative" in L.cc_last_error()
    assert L.cc_debug_fail_alloc(0) == 0
    assert L.cc_measure_peaks(None, None) == -1


def test_label64_and_tuples_reject_bad_arguments_on_host(lib):
    import paper_1607_06156_amd as ccmi
    L = ccmi.lib()
    n = ctypes.c_int64(-5)
    assert L.cc_label64(None, None, -1, 0, None, None, ctypes.byref(n), None) == -1
    assert L.cc_label64(None, None, 0, 0, None, None, ctypes.byref(n), None) == 0 and n.value == 0
    assert L.cc_label64(8, 8, 10, 1 << 31, 8, 8, ctypes.byref(n), None) == -1     # n_max above 2^30
    assert b"2^30" in L.cc_last_error()
    assert L.cc_label64(None, None, 10, 0, 8, 8, ctypes.byref(n), None) == -1     # NULL edges
    st = ccmi.TupleStats()
    assert L.cc_label_tuples(None, None, -1, 5, None, None, 0, ctypes.byref(st)) == -1
    assert L.cc_label_tuples(None, None, 0, 0, None, None, 1, ctypes.byref(st)) == 0
    assert L.cc_label_tuples(8, 8, 1 << 31, 1 << 30, 8, None, 0, ctypes.byref(st)) == -1   # n + 2m + n >= 2^32
    assert L.cc_label_noalloc(None, None, -1, 5, None, None) == -1


def test_router_weights_file_roundtrip(lib, tmp_path):
    import paper_1607_06156_amd as ccmi
    w = np.arange(ccmi.ROUTER_NPARAMS, dtype=np.float32) * 1e-3
    p = tmp_path / "w.txt"
    p.write_text("# test weights\n" + "\n".join(f"{x:.9g}" for x in w) + "\n")
    lib.cc_router_load.argtypes = [ctypes.c_char_p]
    assert lib.cc_router_load(str(p).encode()) == 0
    assert lib.cc_router_loaded() == 1
    bad = tmp_path / "bad.txt"
    bad.write_text("1 2 3\n")
    assert lib.cc_router_load(str(bad).encode()) == -1
    # one line far longer than any line buffer, CRLF ends, a comment in between
    one = tmp_path / "one_line.txt"
    one.write_text("# all on one line\r\n" + " ".join(f"{x:.9g}" for x in w[:-1]) + "\r\n# last\r\n"
                   + f"{w[-1]:.9g}\r\n")
    assert lib.cc_router_load(str(one).encode()) == 0, lib.cc_last_error()
    # a token that is not a finite number is refused, naming it
    for text, word in ((" ".join(["0.5"] * (ccmi.ROUTER_NPARAMS - 1)) + " nan\n", b"nan"),
                       (" ".join(["0.5"] * (ccmi.ROUTER_NPARAMS - 1)) + " 1.5e99\n", b"1.5e99"),
                       ("0.5 0.5x " + " ".join(["0.5"] * (ccmi.ROUTER_NPARAMS - 2)) + "\n", b"0.5x")):
        bad.write_text(text)
        assert lib.cc_router_load(str(bad).encode()) == -1
        assert word in lib.cc_last_error()
    assert lib.cc_router_loaded() == 1          # the weights loaded before stay
    lib.cc_router_set.argtypes = [ctypes.c_void_p]
    assert lib.cc_router_set(None) == 0 and lib.cc_router_loaded() == 0


def test_binding_fails_loudly_without_device_tensors():
    import torch
    import paper_1607_06156_amd as ccmi
    u = torch.zeros(3, dtype=torch.int32)
    with pytest.raises((ValueError, RuntimeError, AssertionError)):
        ccmi.label(u, u, 4, out=torch.empty(4, dtype=torch.int32))
