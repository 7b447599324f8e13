"""Host-side checks of the warm-start network's C-ABI (no GPU needed):
argument validation happens before any device call."""
import ctypes
import os

import pytest

from oracle import convnet as cn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2203_02962_amd", "libfh.so")
pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libfh.so not built")


def test_param_count_matches_the_architecture():
    from paper_2203_02962_amd import fh
    lib = fh.load_library()
    assert lib.fh_net_param_count() == cn.param_count()


@pytest.mark.parametrize("n,batch", [(32, 8), (96, 8), (320, 8), (64, 0), (64, 65)])
def test_create_rejects_bad_sizes(n, batch):
    from paper_2203_02962_amd import fh
    lib = fh.load_library()
    p = ctypes.c_void_p()
    assert lib.fh_net_create(ctypes.byref(p), 0, n, batch) == fh.FH_EINVAL
    assert not p.value


def test_null_arguments_are_rejected():
    from paper_2203_02962_amd import fh
    lib = fh.load_library()
    assert lib.fh_net_create(None, 0, 64, 8) == fh.FH_EINVAL
    assert lib.fh_net_set_params(None, None) == fh.FH_EINVAL
    assert lib.fh_net_forward(None, 1, None, None, None) == fh.FH_EINVAL
    assert lib.fh_net_train(None, 1, None, None, None, 8, 1, None, None, None) == fh.FH_EINVAL
    assert lib.fh_net_last_error(None) == b"null network"
