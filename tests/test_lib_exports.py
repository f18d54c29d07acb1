"""The C-ABI library loads on a machine without a GPU and exports every entry
point its header declares (no compute calls)."""
import ctypes
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cptraj.h")
LIB = os.path.join(ROOT, "paper_2510_25143_amd", "libcptraj.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cpt_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def built():
    if not os.path.exists(LIB):
        from paper_2510_25143_amd import build
        build.build()
    return LIB


def test_header_declares_the_boundary():
    names = declared()
    for n in ["cpt_compress", "cpt_decompress", "cpt_extract_trajectories", "cpt_stream_info",
              "cpt_compress_bound", "cpt_last_error"]:
        assert n in names


def test_library_loads_and_exports_every_declared_symbol(built):
    L = ctypes.CDLL(built)
    for n in declared():
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", built], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (cpt_[a-z_0-9]+)", out))
    assert set(declared()) <= exported


def test_binding_names_match_the_boundary(built):
    import paper_2510_25143_amd as cpt
    for n in cpt.EXPORTS:
        assert n in declared()
    for py in ["compress", "decompress", "extract_trajectories", "stream_info", "verify",
               "field_params", "compress_bound", "compress_debug"]:
        assert callable(getattr(cpt, py))


def test_stream_info_rejects_garbage_on_host(built):
    """cpt_stream_info parses host memory only, so it runs without a GPU."""
    import numpy as np
    import oracle
    import synthfields
    import paper_2510_25143_amd as cpt
    import torch
    f, _ = synthfields.workload(0)
    b = oracle.compress(f.numpy(), 1e-2)
    info = cpt.stream_info(torch.from_numpy(b))
    ref = oracle.stream_info(b)
    for k in ["H", "W", "T", "k", "eps", "K", "R", "total_len", "n_q", "n_raw"]:
        assert info[k] == ref[k]
    bad = b.copy()
    bad[0] ^= 1
    with pytest.raises(cpt.CptError):
        cpt.stream_info(torch.from_numpy(bad))
    with pytest.raises(cpt.CptError):
        cpt.stream_info(torch.from_numpy(b[:100].copy()))


SHORT_STREAMS = r'''
import ctypes, sys
L = ctypes.CDLL(sys.argv[1])
L.cpt_last_error.restype = ctypes.c_char_p
buf = (ctypes.c_uint32 * 64)()          # host memory: never read, every stream is too short
out = (ctypes.c_float * 16)()
P = ctypes.c_void_p
L.cpt_decompress.argtypes = [P, ctypes.c_size_t, P, ctypes.c_size_t, P]
st = L.cpt_decompress(ctypes.addressof(buf), 100, ctypes.addressof(out), 16, None)
msg = L.cpt_last_error().decode()
streams = (P * 2)(ctypes.addressof(buf), ctypes.addressof(buf))
lens = (ctypes.c_size_t * 2)(0, 255)
fields = (P * 2)(ctypes.addressof(out), ctypes.addressof(out))
caps = (ctypes.c_size_t * 2)(16, 16)
status = (ctypes.c_int32 * 2)(7, 7)
L.cpt_decompress_batch.argtypes = [ctypes.c_int, P, P, P, P, P, P]
sb = L.cpt_decompress_batch(2, streams, lens, fields, caps, status, None)
print(st, sb, status[0], status[1], msg)
'''


def test_streams_shorter_than_a_header_touch_no_device(built):
    """As the first calls of a fresh process, decompressing streams that are
    all shorter than the 256-byte header reports a corrupt stream without
    staging, device work or any read of the stream."""
    r = subprocess.run([sys.executable, "-c", SHORT_STREAMS, built], capture_output=True, text=True,
                       env=dict(os.environ, HIP_VISIBLE_DEVICES=""), timeout=120)
    assert r.returncode == 0, r.stderr
    st, sb, s0, s1, *msg = r.stdout.split()
    assert (int(st), int(sb), int(s0), int(s1)) == (-3, -3, -3, -3)
    assert "shorter than its header" in " ".join(msg)


def test_stream_info_reads_a_container_on_host(built):
    """The header of a container of the lossless stage is readable as is."""
    import numpy as np
    import oracle
    import synthfields
    import paper_2510_25143_amd as cpt
    import torch
    f, _ = synthfields.workload(0)
    b = oracle.compress(f.numpy(), 1e-2)
    c = oracle.compress(f.numpy(), 1e-2, backend=1)
    info = cpt.stream_info(torch.from_numpy(c))
    assert info["backend"] == 1 and info["total_len"] == len(b)
    assert cpt.stream_info(torch.from_numpy(b))["backend"] == 0
    bad = c.copy()
    bad[248] ^= 2   # container tag
    with pytest.raises(cpt.CptError):
        cpt.stream_info(torch.from_numpy(bad))
    assert cpt.compress_bound(64, 64, 8) >= oracle.lib().cpo_compress_bound(64, 64, 8)


EXEC_OPTIONS = r'''
import ctypes, sys
L = ctypes.CDLL(sys.argv[1])
L.cpt_last_error.restype = ctypes.c_char_p
P = ctypes.c_void_p
class Ex(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("schedule", ctypes.c_int32), ("group", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("field_tile", ctypes.c_int32),
                ("phase_blocks", ctypes.c_int32)]
buf = (ctypes.c_uint32 * 64)()          # host memory: never read, every call is refused first
fields = (P * 1)(ctypes.addressof(buf))
outs = (P * 1)(ctypes.addressof(buf))
hwt = (ctypes.c_int32 * 3)(16, 16, 2)
caps = (ctypes.c_size_t * 1)(256)
lens = (ctypes.c_size_t * 1)()
status = (ctypes.c_int32 * 1)()
L.cpt_compress_batch.argtypes = [ctypes.c_int, P, P, ctypes.c_double, P, P, P, P, P, P, P]
for size, tile, pb in ((28, 0, 3), (28, 0, -1), (28, 3, 0), (24, 5, 0), (26, 0, 0)):
    ex = Ex(size, 0, 0, 0, 0, tile, pb)
    st = L.cpt_compress_batch(1, fields, hwt, 1e-2, None, ctypes.byref(ex), outs, caps, lens, status, None)
    print(size, tile, pb, st, L.cpt_last_error().decode().replace(" ", "_"))
'''


def test_exec_options_are_checked_on_host(built):
    """Execution options out of range (blocks per phase workgroup, field
    tile) and a struct_size of no known layout are refused before any device
    work, in every layout that holds the field."""
    r = subprocess.run([sys.executable, "-c", EXEC_OPTIONS, built], capture_output=True, text=True,
                       env=dict(os.environ, HIP_VISIBLE_DEVICES=""), timeout=120)
    assert r.returncode == 0, r.stderr
    rows = [line.split() for line in r.stdout.strip().splitlines()]
    assert len(rows) == 5
    want = ["phase_blocks", "phase_blocks", "field_tile", "field_tile", "struct_size"]
    for (size, tile, pb, st, msg), w in zip(rows, want):
        assert int(st) == -1 and w in msg, (size, tile, pb, st, msg)
