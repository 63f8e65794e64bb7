"""The measurement probes (helm_probe_mfma, helm_probe_copy): the copy is bit-exact and refuses
bad arguments; the MFMA loop reports its flop count and leaves finite chain sums."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1107_2461_amd import _lib, load
    return torch, load(), _lib


def test_probe_copy_exact_and_checked(env):
    torch, lib, L = env
    n = (1 << 20) + 48                                  # a ragged tail of three 16-byte values
    src = torch.randint(0, 256, (n,), dtype=torch.uint8, device="cuda")
    dst = torch.zeros(n, dtype=torch.uint8, device="cuda")
    assert lib.helm_probe_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), n, None) == L.HELM_OK
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
    p = src.data_ptr()
    assert lib.helm_probe_copy(C.c_void_p(p), C.c_void_p(dst.data_ptr()), n - 8, None) == L.HELM_EINVAL
    assert lib.helm_probe_copy(C.c_void_p(p + 8), C.c_void_p(dst.data_ptr()), 1024, None) == L.HELM_EINVAL
    assert lib.helm_probe_copy(C.c_void_p(p), C.c_void_p(p + 512), 1024, None) == L.HELM_EINVAL


@pytest.mark.parametrize("kind,per_mfma", [(0, 2 * 16 * 16 * 32), (1, 2 * 16 * 16 * 4), (2, 2 * 16 * 16 * 4)])
def test_probe_mfma_flops_and_output(env, kind, per_mfma):
    torch, lib, L = env
    blocks, iters = 8, 4
    out = torch.full((blocks * 256,), float("nan"), dtype=torch.float32, device="cuda")
    for chains in (4, 8, 16):
        fl = C.c_double()
        assert lib.helm_probe_mfma(kind, chains, iters, blocks, C.c_void_p(out.data_ptr()), None,
                                   C.byref(fl)) == L.HELM_OK
        torch.cuda.synchronize()
        assert fl.value == per_mfma * chains * iters * blocks * 4
        o = out.cpu().numpy()
        assert np.isfinite(o).all() and (o > 0).all()
    assert lib.helm_probe_mfma(kind, 5, iters, blocks, C.c_void_p(out.data_ptr()), None, None) == L.HELM_EINVAL
    assert lib.helm_probe_mfma(3, 4, iters, blocks, C.c_void_p(out.data_ptr()), None, None) == L.HELM_EINVAL
