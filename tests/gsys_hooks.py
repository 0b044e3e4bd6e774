"""ctypes binding of the test-only hook library (tests/native/libgsys_testing.so,
built by the package build next to its source): host threads that speak
the GPU's slot protocol, raw calls, fault injection and ring views."""
import ctypes as C
import os

import paper_1705_06965_amd as g  # loads libgsys.so first (the hooks link to it)

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "native",
                        "libgsys_testing.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libgsys_testing.so is not built: run __graft_entry__.build()")
lib = C.CDLL(LIB_PATH)

EMU_BLOCKING, EMU_LIST = 0x1, 0x2

_P = C.c_void_p
for name, (res, args) in {
    "gsys_test_emulate": (C.c_int, [_P, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32, C.c_int,
                                    C.c_uint64, C.c_uint64, C.c_uint32, _P, _P, C.c_uint64]),
    "gsys_test_raw_call": (C.c_int, [_P, C.c_uint16, C.c_uint8, _P, _P, C.c_uint64]),
    "gsys_test_claim_only": (C.c_int64, [_P, C.c_uint32]),
    "gsys_test_ring_ctl": (C.c_int, [_P, _P, C.c_uint64]),
    "gsys_test_inject": (C.c_int, [_P, C.c_uint16, C.c_int32, C.c_uint32]),
    "gsys_test_unregister_now": (C.c_int, [_P, C.c_uint32]),
}.items():
    f = getattr(lib, name)
    f.restype = res
    f.argtypes = args


def declared():
    """Names of the C functions native/gsys_testing.h declares."""
    import re
    with open(os.path.join(os.path.dirname(LIB_PATH), "gsys_testing.h")) as fh:
        return re.findall(r"^\w[\w\s\*]*?\b(gsys_\w+)\s*\(", fh.read(), re.M)
