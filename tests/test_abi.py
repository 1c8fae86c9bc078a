"""CPU checks of the C ABI: the library loads and exports every declared symbol."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "wdf.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wdf_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ["wdf_create", "wdf_model_load", "wdf_background_load", "wdf_explain", "wdf_base_value",
              "wdf_debug_patterns", "wdf_debug_histograms", "wdf_debug_tables", "wdf_server_create",
              "wdf_server_submit", "wdf_server_wait", "wdf_server_stats", "wdf_last_error"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2511_09376_amd import wdf
    if not os.path.exists(wdf.LIB_PATH):
        pytest.skip("libwdf.so not built")
    lib = ctypes.CDLL(wdf.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"missing exports: {missing}"
    assert set(wdf.EXPORTS) == set(declared_functions())
    assert wdf.lib().wdf_last_error() == b""


def test_binding_types_follow_the_header():
    """Every declared function has its argument count and return width in the
    binding (a 64-bit return read as int would truncate sizes)."""
    from paper_2511_09376_amd import wdf
    if not os.path.exists(wdf.LIB_PATH):
        pytest.skip("libwdf.so not built")
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    L = wdf.lib()
    decls = re.findall(r"^\s*((?:const\s+)?[a-z_0-9]+(?:\s*\*)?)\s*(wdf_[a-z_]+)\s*\(([^)]*)\)\s*;", text, flags=re.M)
    assert {n for _, n, _ in decls} == set(declared_functions())
    for ret, name, args in decls:
        fn = getattr(L, name)
        n_args = 0 if args.strip() in ("", "void") else args.count(",") + 1
        assert fn.argtypes is not None and len(fn.argtypes) == n_args, name
        ret = ret.replace(" ", "")
        if ret == "int64_t":
            assert fn.restype is ctypes.c_int64, name
        elif ret == "int":
            assert fn.restype in (ctypes.c_int, None) or fn.restype is ctypes.c_int32, name
        elif ret == "void":
            assert fn.restype in (None, ctypes.c_int), name
        elif ret == "constchar*":
            assert fn.restype is ctypes.c_char_p, name


def test_product_path_does_not_touch_the_oracle():
    pkg = os.path.join(ROOT, "paper_2511_09376_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "woodelf_oracle" not in src, f


def test_missing_library_fails_loudly():
    """Without libwdf.so every entry point raises: there is no fallback path."""
    import subprocess
    import sys
    code = ("import paper_2511_09376_amd.wdf as w\n"
            "w.LIB_PATH = '/nonexistent/libwdf.so'\n"
            "from paper_2511_09376_amd import synth\n"
            "for call in (lambda: w.Context(0), lambda: w.specialised_source(synth.WORKLOADS['small'].ensemble())):\n"
            "    try:\n"
            "        call()\n"
            "    except ImportError as e:\n"
            "        assert 'is missing' in str(e)\n"
            "    else:\n"
            "        raise SystemExit('no error')\n"
            "print('refused')\n")
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert res.returncode == 0 and res.stdout.strip() == "refused", res.stderr


def test_handles_left_open_at_exit_close_quietly():
    """Handles still referenced when the interpreter exits on an uncaught
    error (torch imported, so the module teardown order is torch's) are
    destroyed without an error from their finalizers."""
    import subprocess
    import sys
    code = ("import torch\n"
            "from paper_2511_09376_amd import wdf\n"
            "objs = []\n"
            "for cls in (wdf.Context, wdf.Model, wdf.Background, wdf.Graph, wdf.Server):\n"
            "    o = cls.__new__(cls)\n"
            "    o.h = None\n"
            "    objs.append(o)\n"
            "a, b, c, d, e = objs\n"
            "def fail():\n"
            "    raise ValueError('planned')\n"
            "fail()\n")
    res = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=300)
    assert res.returncode == 1 and "ValueError: planned" in res.stderr
    assert "Exception ignored" not in res.stderr, res.stderr
