"""The C ABI library loads on a machine without a GPU, exports every function include/hisq.h
declares, and rejects bad arguments before touching a device."""
import ctypes

import pytest

from paper_1409_1510_amd import hisq


def test_exports_every_declared_symbol():
    names = hisq.header_functions()
    assert len(names) >= 12
    lib = ctypes.CDLL(hisq.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_header_constants_match_binding():
    text = open(hisq.HEADER_PATH).read()
    for name in ("HISQ_OK", "HISQ_ERR_ARG", "HISQ_ERR_STATE", "HISQ_ERR_HIP", "HISQ_ERR_OOM",
                 "HISQ_ERR_NOCONV", "HISQ_ERR_NONFINITE", "HISQ_F64", "HISQ_F32", "HISQ_F16",
                 "HISQ_CG_F64", "HISQ_CG_MIXED", "HISQ_FCG_NN", "HISQ_LINKS_ALL"):
        assert name in text
    assert "#define HISQ_MAX_RHS 64" in text and hisq.HISQ_MAX_RHS == 64


@pytest.mark.parametrize("dims", [(4, 4, 4, 5), (2, 4, 4, 4), (4, 4, 4, 3), (0, 4, 4, 4)])
def test_create_rejects_bad_extents(dims):
    with pytest.raises(hisq.HisqError) as e:
        hisq.hisq_create(dims, 0, 0)
    assert e.value.code == hisq.HISQ_ERR_ARG
    assert "extent" in hisq.hisq_last_error(None)


def test_null_context_is_rejected():
    lib = hisq.library()
    assert lib.hisq_destroy(None) == hisq.HISQ_OK
    assert lib.hisq_dslash_mrhs(None, 1, 0, 1, None, None) == hisq.HISQ_ERR_ARG
    assert lib.hisq_apply_m(None, 0, 0.1, 1, None, None, None) == hisq.HISQ_ERR_ARG
    assert lib.hisq_dot_mrhs(None, 0, 1, None, None, None) == hisq.HISQ_ERR_ARG
    assert lib.hisq_dot_mrhs_noalloc(None, 0, 1, None, None, None) == hisq.HISQ_ERR_ARG
    assert lib.hisq_load_links(None, None, None, 7, 18) == hisq.HISQ_ERR_ARG
    assert lib.hisq_cg_mrhs(None, 0.1, 1, None, None, None, None) == hisq.HISQ_ERR_ARG
    assert lib.hisq_set_launch(None, 0, 1, None) == hisq.HISQ_ERR_ARG
    assert lib.hisq_autotune(None, 0, 1, 0, None, None) == hisq.HISQ_ERR_ARG


def test_one_hip_runtime_per_process():
    """libhisq binds to PyTorch's HIP runtime even when imported before torch (two runtimes in
    one process do not share the GPU)."""
    import subprocess
    import sys
    code = ("import sys; sys.path.insert(0, %r)\n"
            "from paper_1409_1510_amd import hisq\n"
            "import torch\n"
            "libs = {l.split()[-1] for l in open('/proc/self/maps') if 'libamdhip64' in l}\n"
            "print(len(libs))\n") % (hisq.os.path.dirname(hisq._HERE),)
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "1"
