"""The C-ABI library loads and exports every function include/hot.h declares
(no device calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hot.h")
LIB = os.path.join(ROOT, "paper_1911_07913_amd", "libhot.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:hot_status|void|double|const char\*)\s+(hot_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("hot_init_scene", "hot_step", "hot_read_particles", "hot_destroy_scene",
                     "hot_scene_footprint", "hot_batch_add", "hot_batch_poll"):
        assert required in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhot.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name
    from paper_1911_07913_amd import hot
    assert set(hot.EXPORTS) == set(declared_functions())


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhot.so not built")
def test_struct_layouts_match_header_sizes():
    from paper_1911_07913_amd import hot
    # hot_params: 8 + 12 + 24 + 24 + 8*3 + 4*5 + 4*3 (+ padding) ; checked against
    # the offsets the C compiler uses for the same declaration
    src = r'''
    #include <stddef.h>
    #include "hot.h"
    size_t sz_params(void){return sizeof(hot_params);}
    size_t sz_stats(void){return sizeof(hot_step_stats);}
    size_t sz_bc(void){return sizeof(hot_bc);}
    size_t sz_mat(void){return sizeof(hot_material);}
    size_t off_precision(void){return offsetof(hot_params, precision);}
    size_t off_ms(void){return offsetof(hot_step_stats, ms_prepare);}
    size_t sz_result(void){return sizeof(hot_batch_result);}
    size_t off_msg(void){return offsetof(hot_batch_result, message);}
    '''
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        so = os.path.join(d, "t.so")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-shared", "-fPIC", "-I", os.path.join(ROOT, "include"), c, "-o", so])
        t = ctypes.CDLL(so)
        for f in ("sz_params", "sz_stats", "sz_bc", "sz_mat", "off_precision", "off_ms", "sz_result",
                  "off_msg"):
            getattr(t, f).restype = ctypes.c_size_t
        assert t.sz_params() == ctypes.sizeof(hot.hot_params)
        assert t.sz_stats() == ctypes.sizeof(hot.hot_step_stats)
        assert t.sz_bc() == ctypes.sizeof(hot.hot_bc)
        assert t.sz_mat() == ctypes.sizeof(hot.hot_material)
        assert t.off_precision() == hot.hot_params.precision.offset
        assert t.off_ms() == hot.hot_step_stats.ms_prepare.offset
        assert t.sz_result() == ctypes.sizeof(hot.hot_batch_result)
        assert t.off_msg() == hot.hot_batch_result.message.offset
