"""Saved systems: the header reader (host only) against handcrafted files, and
the struct layout against the header. The device round trips are in
tests/test_gpu_persist.py."""
import ctypes
import os
import struct

import pytest

import paper_1912_01491_amd as lb

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header(kind=0, N=5, M=None, nnz=0, magic=b"LBSYSTEM", version=1, h=0):
    M = N * N - 1 if M is None else M
    return magic + struct.pack("<IIqqqQ4Q", version, kind, N, M, nnz, h, 0, 0, 0, 0)


def info(path):
    s = lb._System()
    rc = lb.load().lindblad_load_system_info(str(path).encode(), ctypes.byref(s))
    return rc, s


def test_header_is_80_bytes():
    assert len(header()) == 80


def test_info_reads_a_valid_header(tmp_path):
    p = tmp_path / "ok.bin"
    p.write_bytes(header(kind=1, N=7, nnz=123) + b"\0" * 16)
    rc, s = info(p)
    assert rc == 0 and (s.kind, s.N, s.nnz) == (1, 7, 123)
    assert lb.load_system_info(str(p)) == (1, 7, 123)


@pytest.mark.parametrize("data", [
    header(magic=b"NOTASYS!"),
    header(version=2),
    header(M=10),                 # M != N^2 - 1
    header(kind=3),
    header(kind=0, nnz=5),        # dense files carry no nnz
    header(N=1),
    header()[:40],                # truncated
])
def test_info_rejects_bad_headers(tmp_path, data):
    p = tmp_path / "bad.bin"
    p.write_bytes(data)
    rc, _ = info(p)
    assert rc == -8
    assert lb.load().lb_last_error()


def test_info_missing_file(tmp_path):
    rc, _ = info(tmp_path / "nope.bin")
    assert rc == -8


def test_system_struct_layout_matches_header(tmp_path):
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    src = tmp_path / "sys.c"
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "lindblad.h"\n'
                   'int main(void) { printf("%zu %zu %zu %zu %zu %zu\\n", sizeof(lb_system), '
                   'offsetof(lb_system, ldq), offsetof(lb_system, nnz), offsetof(lb_system, Q), '
                   'offsetof(lb_system, val), offsetof(lb_system, K)); return 0; }\n')
    exe = tmp_path / "sys"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(x) for x in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    S = lb._System
    assert got == [ctypes.sizeof(S), S.ldq.offset, S.nnz.offset, S.Q.offset, S.val.offset, S.K.offset]
