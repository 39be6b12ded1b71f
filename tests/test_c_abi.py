"""The C ABI used from C and C++ programs (no GPU): include/fewbody.h
compiles as C99 and as C++17 with warnings as errors, links against
libfewbody.so, and the host-side calls behave as documented."""
import ctypes
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1208_1157_amd")
SRC = os.path.join(ROOT, "tests", "c", "abi_check.c")


def build_and_run(tmp_path, compiler, std, lang):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    if not os.path.exists(os.path.join(PKG, "libfewbody.so")):
        pytest.skip("libfewbody.so is not built")
    exe = str(tmp_path / f"abi_check_{compiler}")
    cmd = [compiler, f"-std={std}", "-Wall", "-Wextra", "-pedantic", "-Werror", *lang,
           "-I", os.path.join(ROOT, "include"), SRC, "-L", PKG, "-lfewbody", f"-Wl,-rpath,{PKG}",
           "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True, timeout=120).stdout
    return dict(line.split(" ", 1) for line in out.strip().splitlines())


@pytest.mark.parametrize("compiler,std,lang", [("gcc", "c99", []), ("g++", "c++17", ["-x", "c++"])])
def test_header_compiles_links_and_validates(tmp_path, compiler, std, lang):
    r = build_and_run(tmp_path, compiler, std, lang)
    assert r["version_has_gfx950"] == "1"
    assert r["opts_default"].split() == ["0", "0.01", "0", "100", "0"]
    assert r["workspace_ok"] == "1" and r["workspace_bad"] == "0"
    assert int(r["log_rv"]) == 8 * 4 * 2 * 3
    assert int(r["log_state"]) == 8 * 4 * (3 + 6 * (3 + 5 + 40))
    assert r["log_bad_kind"] == "0"
    assert r["integrate_null"] == "-1" and r["last_error_set"] == "1"
    assert r["create_bad_n"] == "-1 1"
    assert r["server_request_ok"] == "1"
    assert r["server_request_large"] == "0"      # the server takes at most 16 bodies per system
    assert r["server_bad_spread"] == "0"
    # the C structs and the binding's ctypes mirrors agree
    from paper_1208_1157_amd import fewbody as fbmod
    assert r["sizes"].split() == [str(ctypes.sizeof(fbmod.FbServerOpts)),
                                  str(ctypes.sizeof(fbmod.FbServerStats))]
