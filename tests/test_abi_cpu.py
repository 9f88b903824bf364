"""The C ABI on a machine without a GPU: the library loads, exports every
function include/rsi.h declares, and rejects bad arguments before touching
the GPU.  No compute call is made here."""
import ctypes
import os
import re

import pytest
import torch

import paper_2305_01867_amd as rsi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "rsi.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsi_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    names = declared_functions()
    assert "rsi_build" in names and "rsi_intersect" in names and len(names) >= 9
    L = ctypes.CDLL(rsi.library_path)
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing


def test_abi_version_and_status_strings():
    L = rsi.lib()
    assert L.rsi_abi_version() == 7
    for code in range(7):
        assert L.rsi_status_string(code).decode().startswith("RSI_")
    assert b"unknown" in L.rsi_status_string(99)


def _build(vp, nv, fp, nt, opts=None, out=True):
    L = rsi.lib()
    h = ctypes.c_void_p()
    return L.rsi_build(vp, nv, fp, nt, opts, None, ctypes.byref(h) if out else None)


def test_build_argument_errors_need_no_gpu():
    L = rsi.lib()
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert _build(p, 3, p, 1, out=False) == 1               # out is NULL
    assert _build(None, 3, p, 1) == 1                       # NULL vertices
    assert _build(p, 3, None, 1) == 1                       # NULL triangles
    assert _build(p, -1, p, 1) == 1                         # negative count
    assert _build(p, 3, p, -5) == 1
    assert _build(p, 3, p, 1 << 30) == 6                    # capacity
    odd = ctypes.c_void_p(ctypes.addressof(buf) + 1)
    assert _build(odd, 3, p, 1) == 1                        # misaligned
    bad = rsi._BuildOpts(31, 0)
    assert _build(p, 3, p, 1, ctypes.byref(bad)) == 1       # morton_bits
    assert b"morton_bits" in L.rsi_last_error()


def test_intersect_argument_errors_need_no_gpu():
    L = rsi.lib()
    outs = rsi._Outputs()
    # NULL / bogus handle
    assert L.rsi_intersect(None, None, None, 0, 0, None, ctypes.byref(outs), None) == 5
    assert L.rsi_intersect_noalloc(None, None, None, 0, 0, None, ctypes.byref(outs), None) == 5
    assert L.rsi_destroy(None) == 0
    assert L.rsi_mesh_info_get(None, None) == 5
    assert L.rsi_mesh_export(None, 0, None, 0, None) == 5


def test_debug_certify_argument_errors_need_no_gpu():
    L = rsi.lib()
    assert L.rsi_debug_certify(None, None, None, -1, None, None, None) == 1  # negative count
    assert L.rsi_debug_certify(None, None, None, 0, None, None, None) == 0   # nothing to do
    assert L.rsi_debug_certify(None, None, None, 5, None, None, None) == 1   # NULL arrays
    assert b"non-NULL" in L.rsi_last_error()


def test_derived_output_argument_errors_need_no_gpu():
    L = rsi.lib()
    assert L.rsi_derive(None, None, -1, None, None, None, None, None) == 1
    assert L.rsi_derive(None, None, 4, None, None, None, None, None) == 1   # NULL inputs
    assert L.rsi_compact_hits(None, None, -1, None, None, None, None, None, None, None, None) == 1
    assert L.rsi_compact_hits(None, None, 4, None, None, None, None, None, None, None, None) == 1


def test_valid_arguments_without_a_gpu_report_state_error():
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    buf = ctypes.create_string_buffer(64)
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert _build(p, 3, p, 1) == 5
    assert rsi.lib().rsi_last_error()


def test_python_wrapper_refuses_int64_indices_and_host_tensors():
    V = torch.zeros((3, 3), dtype=torch.float32)
    with pytest.raises(TypeError):
        rsi.rsi_build(V, torch.zeros((1, 3), dtype=torch.int64))
    with pytest.raises(ValueError):
        rsi.rsi_build(V, torch.zeros((1, 3), dtype=torch.int32))   # not on the GPU
    with pytest.raises(TypeError):
        rsi.rsi_build(V.double(), torch.zeros((1, 3), dtype=torch.int32))


def test_stream_copy_argument_errors_need_no_gpu():
    L = rsi.lib()
    assert L.rsi_stream_copy(None, None, 0, None) == 0      # nothing to copy
    assert L.rsi_stream_copy(None, None, -16, None) == 1    # negative size
    assert L.rsi_stream_copy(None, None, 24, None) == 1     # not a multiple of 16
    assert L.rsi_stream_copy(None, None, 32, None) == 1     # NULL buffers
    assert b"16-byte" in L.rsi_last_error()


def test_export_codes_are_distinct():
    text = open(os.path.join(ROOT, "include", "rsi.h")).read()
    codes = {m.group(1): int(m.group(2)) for m in re.finditer(r"\b(RSI_EXPORT_[A-Z_]+)\s*=\s*(\d+)", text)}
    codes.update({m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(RSI_EXPORT_[A-Z_]+)\s+(\d+)", text)})
    assert "RSI_EXPORT_MESH_ROOTS" in codes and len(codes) >= 10
    assert len(set(codes.values())) == len(codes), codes
    assert codes == {k.upper().join(("RSI_EXPORT_", "")): v for k, v in rsi.EXPORTS.items()}
