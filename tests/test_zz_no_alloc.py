"""The allocation-free check (cpt_verify_noalloc, called through the C ABI)
gives the same false-case counts, maximum error and PSNR as cpt_verify, bit
for bit, on two calls in a row with the second field smaller than the first
(the shared scratch array keeps the first call's contents), and refuses a
field beyond its fixed scratch size before any device work."""
import ctypes

import numpy as np
import pytest
import torch

import synthfields

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cpt():
    import paper_2510_25143_amd as m
    m.lib()
    assert torch.cuda.is_available()
    return m


def pair(shape, seed, sigma):
    rng = np.random.default_rng(seed)
    f, _ = synthfields.workload(0, shape=shape)
    a = f.numpy()
    b = a + rng.normal(0, sigma, a.shape).astype(np.float32)
    return torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()


def call_noalloc(cpt, a, b, k):
    _, T, H, W = a.shape
    r = cpt.VerifyResult()
    st = cpt.lib().cpt_verify_noalloc(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), H, W, T, k,
                                      ctypes.byref(r), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == cpt.OK, cpt.lib().cpt_last_error()
    return dict(fc_t=r.fc_t, fc_s=r.fc_s, max_err=r.max_err, psnr=r.psnr)


def test_noalloc_check_matches_cpt_verify(cpt):
    cases = [((160, 200, 9), 1, 0.02), ((40, 56, 4), 2, 0.01)]   # second call smaller
    for shape, seed, sigma in cases:
        a, b = pair(shape, seed, sigma)
        k, _, _ = cpt.field_params(a, 1e-2)
        want = cpt.verify(a, b, k)
        got = call_noalloc(cpt, a, b, k)
        assert got == want, (shape, got, want)
        assert want["fc_t"] > 0 and want["fc_s"] > 0
        same = call_noalloc(cpt, a, a.clone(), k)
        assert (same["fc_t"], same["fc_s"], same["max_err"]) == (0, 0, 0.0)


def test_noalloc_check_refuses_fields_beyond_its_scratch(cpt):
    a = torch.zeros((2, 1, 2, 2), dtype=torch.float32, device="cuda")
    r = cpt.VerifyResult()
    H, W = 2048, 2048
    T = cpt.VERIFY_NOALLOC_MAX_VERTICES // (H * W) + 1
    st = cpt.lib().cpt_verify_noalloc(ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(a.data_ptr()), H, W, T, 0,
                                      ctypes.byref(r), ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert st == cpt.EUNSUPPORTED
    assert "at most %d vertices" % cpt.VERIFY_NOALLOC_MAX_VERTICES in cpt.lib().cpt_last_error().decode()
