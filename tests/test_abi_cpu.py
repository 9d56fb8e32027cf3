"""CPU checks of the C ABI: the library loads, exports every function the
header declares, the Python binding wraps each of them, and calls that need
no device reject bad arguments.  No kernel is launched here."""
import ctypes as C
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = glob.glob(os.path.join(ROOT, "include", "*.h"))
DECL = re.compile(r"^\s*(?:mbmd_status|void|const\s+char\s*\*)\s*\*?\s*(mbmd_\w+)\s*\(", re.M)


def declared():
    names = []
    for h in HEADERS:
        names += DECL.findall(open(h).read())
    return names


def test_header_declares_the_boundary():
    names = declared()
    for must in ("mbmd_create", "mbmd_destroy", "mbmd_set_tersoff", "mbmd_set_sw",
                 "mbmd_neighbors", "mbmd_compute", "mbmd_nve_run", "mbmd_workspace_size",
                 "mbmd_bind_workspace"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1610_03343_amd as mb
    lib = C.CDLL(mb.LIB_PATH)
    for name in declared():
        assert hasattr(lib, name), name
    # and the binding sets a signature for each
    for name in declared():
        assert getattr(mb.lib(), name).argtypes is not None or name == "mbmd_destroy", name


def test_null_context_rejected_without_device():
    import paper_1610_03343_amd as mb
    lib = mb.lib()
    p = mb.tersoff_struct(__import__("workload").TERSOFF_SI_1989)
    assert lib.mbmd_set_tersoff(None, C.byref(p)) == mb.MBMD_EINVAL
    assert lib.mbmd_set_neighbor(None, 0.5, 16) == mb.MBMD_EINVAL
    sz = C.c_size_t()
    assert lib.mbmd_workspace_size(None, 10, C.byref(sz)) == mb.MBMD_EINVAL
    assert lib.mbmd_compute(None, 0, 0, None, None, None, None, None, None, None, None) == mb.MBMD_EINVAL
    assert lib.mbmd_last_error(None) == b"null context"
    lib.mbmd_destroy(None)
    assert lib.mbmd_create(None, 0, None) == mb.MBMD_EINVAL


def test_create_reports_device_state():
    """With no HIP device the call fails cleanly with MBMD_EDEVICE."""
    import paper_1610_03343_amd as mb
    h = C.c_void_p()
    st = mb.lib().mbmd_create(C.byref(h), 0, None)
    assert st in (mb.MBMD_OK, mb.MBMD_EDEVICE)
    if st == mb.MBMD_OK:
        mb.lib().mbmd_destroy(h)
    else:
        assert not h.value
    assert mb.lib().mbmd_create(C.byref(h), -1, None) == mb.MBMD_EDEVICE


def test_binding_rejects_cpu_tensors():
    import pytest
    import torch
    import paper_1610_03343_amd as mb
    with pytest.raises(TypeError):
        mb._dptr(torch.zeros(3, 4, dtype=torch.float64), (3, 4), "pos")
