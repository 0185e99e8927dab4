"""The C-ABI library loads and exports every function declared in
include/ptrom.h, and the Python binding knows every one of them (CPU only:
no compute call is made)."""
import ctypes
import os
import re

from paper_2103_01983_amd import native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "ptrom.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ptrom_[a-z0-9_]+)\s*\(", src)))


def test_header_declares_the_surface():
    names = declared()
    assert "ptrom_velocity" in names and "ptrom_rom_run" in names and len(names) >= 25


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(native.LIB_PATH)
    missing = [n for n in declared() if not hasattr(L, n)]
    assert not missing, missing


def test_binding_covers_every_declared_symbol():
    assert sorted(native.SIGNATURES) == declared()
    native.lib()
    assert native.lib().ptrom_version() == 10000


def test_no_device_create_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        return
    h = ctypes.c_void_p()
    assert native.lib().ptrom_create(ctypes.byref(h), 0) != 0


def test_struct_layouts_match_the_header(tmp_path):
    # every public struct: size and field offsets as a C compiler lays them
    # out from include/ptrom.h, against the binding's ctypes mirrors
    import subprocess
    mirrors = {"ptrom_newton_opts": native.NewtonOpts, "ptrom_newton_stats": native.NewtonStats,
               "ptrom_rom_desc": native.RomDesc}
    src = open(os.path.join(ROOT, "include", "ptrom.h")).read()
    assert set(re.findall(r"\}\s*(ptrom_[a-z0-9_]+)\s*;", src)) == set(mirrors)
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ptrom.h"', "int main(void) {"]
    for cname, cls in mirrors.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    c = tmp_path / "layout.c"
    c.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), "-o", str(exe), str(c)])
    got = {}
    for ln in subprocess.check_output([str(exe)], text=True).splitlines():
        cname, field, val = ln.split()
        got[(cname, field)] = int(val)
    for cname, cls in mirrors.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)


def test_binding_argument_counts_match_the_header():
    # every declared function: the number of C parameters equals the number
    # of ctypes argument types the binding passes
    src = open(os.path.join(ROOT, "include", "ptrom.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    decls = dict(re.findall(r"\b(ptrom_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", src, flags=re.S))
    assert set(decls) == set(native.SIGNATURES)
    for name, params in decls.items():
        params = " ".join(params.split())
        n = 0 if params in ("", "void") else params.count(",") + 1
        assert n == len(native.SIGNATURES[name][1]), (name, n, len(native.SIGNATURES[name][1]))


def test_binding_argument_types_match_the_header():
    # scalar parameters by width and kind, pointers as pointers
    src = open(os.path.join(ROOT, "include", "ptrom.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    decls = dict(re.findall(r"\b(ptrom_[a-z0-9_]+)\s*\(([^;{]*?)\)\s*;", src, flags=re.S))
    scalar = {"float": ctypes.c_float, "double": ctypes.c_double, "int": ctypes.c_int, "int32_t": ctypes.c_int32,
              "int64_t": ctypes.c_int64, "uint32_t": ctypes.c_uint32, "uint64_t": ctypes.c_uint64,
              "size_t": ctypes.c_size_t}
    for name, params in decls.items():
        params = " ".join(params.split())
        if params in ("", "void"):
            continue
        for k, p in enumerate(params.split(",")):
            words = p.replace("*", " * ").split()
            ct = native.SIGNATURES[name][1][k]
            if "*" in words or words[0] == "ptrom_stream":
                assert ct in (ctypes.c_void_p, ctypes.c_char_p) or hasattr(ct, "_type_") and issubclass(
                    ct, ctypes._Pointer), (name, p, ct)
            else:
                base = [w for w in words[:-1] if w != "const"]
                assert len(base) == 1 and base[0] in scalar, (name, p)
                want = scalar[base[0]]
                assert ctypes.sizeof(ct) == ctypes.sizeof(want) and (ct in (ctypes.c_float, ctypes.c_double)) == (
                    want in (ctypes.c_float, ctypes.c_double)), (name, p, ct)
