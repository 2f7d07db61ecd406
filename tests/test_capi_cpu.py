"""Host-side checks of the C ABI (no GPU needed).

* libdwos.so loads and exports every entry point declared in include/dwos.h.
* The ctypes mirrors of the public structs have the C layout (sizes and field
  offsets compiled from the header with g++).
* Without a GPU, dwos_create reports DWOS_EDEVICE instead of crashing.
"""
import ctypes as C
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dwos.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^(?:dwos_status|const char\*|int32_t|void)\s+(dwos_\w+)\s*\(", txt, re.M)))


def test_library_exports_every_declared_symbol():
    from paper_2405_12964_amd import capi
    L = capi.lib()
    names = declared()
    assert len(names) >= 18
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(names) == set(capi.EXPORTED)


def test_struct_layout_matches_header():
    from paper_2405_12964_amd import capi
    src = r'''
#include <cstdio>
#include <cstddef>
#include "dwos.h"
int main() {
  std::printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n", sizeof(dwos_problem), sizeof(dwos_bc), sizeof(dwos_stats),
    offsetof(dwos_problem, src_c0), offsetof(dwos_problem, gauss), offsetof(dwos_problem, n_labels),
    offsetof(dwos_problem, bc), offsetof(dwos_stats, walk_ms), sizeof(dwos_quad), offsetof(dwos_quad, A));
}
'''
    d = tempfile.mkdtemp()
    f = os.path.join(d, "layout.cpp")
    open(f, "w").write(src)
    exe = os.path.join(d, "layout")
    subprocess.check_call(["g++", "-std=c++17", "-I", os.path.dirname(HEADER), "-o", exe, f])
    vals = [int(v) for v in subprocess.check_output([exe]).split()]
    P, S = capi.dwos_problem, capi.dwos_stats
    Q = capi.dwos_quad
    assert vals == [C.sizeof(P), C.sizeof(capi.dwos_bc), C.sizeof(S), P.src_c0.offset, P.gauss.offset,
                    P.n_labels.offset, P.bc.offset, S.walk_ms.offset, C.sizeof(Q), Q.A.offset]


def test_create_without_gpu_reports_device_error():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2405_12964_amd import capi
    ctx = C.c_void_p()
    rc = capi.dwos_create(3, capi.DWOS_FP32, None, C.byref(ctx))
    assert rc == capi.DWOS_EDEVICE
    assert ctx.value is None
    assert capi.dwos_last_error()  # message set
    assert capi.dwos_create(4, capi.DWOS_FP32, None, C.byref(ctx)) == capi.DWOS_EINVAL
    assert capi.dwos_destroy(None) == capi.DWOS_OK
    # the control-variate network needs a device too
    m = C.c_void_p()
    B = (C.c_float * 32)()
    assert capi.dwos_mlp_create(2, 16, B, None, C.byref(m)) == capi.DWOS_EDEVICE
    assert m.value is None
    assert capi.dwos_mlp_create(2, 40, B, None, C.byref(m)) == capi.DWOS_EINVAL
    assert capi.dwos_mlp_theta_size() == 4 * (64 * 64 + 64) + 65
    assert capi.dwos_cv_attach(None, None, 1.0) == capi.DWOS_EINVAL


def test_missing_library_fails_loudly(tmp_path, monkeypatch):
    """No fallback: without libdwos.so the binding raises instead of
    computing anything elsewhere."""
    from paper_2405_12964_amd import capi
    monkeypatch.setattr(capi, "_lib", None)
    monkeypatch.setattr(capi, "LIB_PATH", str(tmp_path / "libdwos.so"))
    with pytest.raises(ImportError):
        capi.lib()
