"""log_likelihood_batch_noalloc (the entry point that allocates nothing: its
scratch is a file-scope device array of the library) against
log_likelihood_batch, through the C ABI: two calls in a row, the second with
fewer items, at the benchmark's 128 x 128 FP32 tile and at 64 x 64 FP64;
the calls' misfits, status and CG iterations must equal the allocating
entry point's bit for bit (the same kernels on the same items)."""
import ctypes

import numpy as np
import pytest

import oracle
from gpu_common import THETA_TRUE, TAU, make_problem, need_gpu, theta_batch
from paper_1605_04718_amd import inputs

pytestmark = pytest.mark.gpu


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def noalloc(p, th):
    """Calls the C entry point directly (ctypes): phi, status, iterations."""
    import torch
    from paper_1605_04718_amd import _lib
    n = th.shape[0]
    phi = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
    st = torch.full((n,), -7, dtype=torch.int32, device="cuda")
    it = torch.full((n, 2), -7, dtype=torch.int32, device="cuda")
    code = _lib.lib().log_likelihood_batch_noalloc(p.h, n, _ptr(th), _ptr(phi), _ptr(st), _ptr(it),
                                                   None)
    _lib.check(code, "log_likelihood_batch_noalloc")
    return phi, st, it


@pytest.mark.parametrize("n, steps, precision, m1, m2",
                         [(128, 40, 0, 300, 37), (64, 30, 1, 90, 11), (128, 8, 1, 70, 9)])
def test_noalloc_matches_the_allocating_entry_point(n, steps, precision, m1, m2):
    import torch
    need_gpu()
    u0, v0 = inputs.initial_fields(n, THETA_TRUE[0], THETA_TRUE[1])
    uo, _, _, _ = oracle.forward_solve(THETA_TRUE, u0, v0, TAU, steps, rtol=1e-12)
    y, sigma = inputs.noisy_data(uo, 0.01)
    p, _, _ = make_problem(n, steps, precision=precision, y=y, sigma=sigma, u0=u0, v0=v0,
                           max_batch=m1)
    for m, seed in ((m1, 71), (m2, 72)):
        th = torch.tensor(np.vstack([THETA_TRUE, theta_batch(m - 1, seed=seed)]), device="cuda")
        print(f"noalloc n={n} precision={precision}: {m} items", flush=True)
        phi_a, st_a, it_a = noalloc(p, th)
        phi_b, st_b, it_b = p.log_likelihood(th)
        torch.cuda.synchronize()
        assert torch.equal(st_a, st_b)
        assert torch.equal(it_a, it_b)
        assert np.array_equal(phi_a.cpu().numpy(), phi_b.cpu().numpy())
        assert int((st_a == 0).sum()) > m // 2
    p.close()


def test_noalloc_rejects_what_it_does_not_serve():
    import torch
    from paper_1605_04718_amd import _lib
    need_gpu()
    p, _, _ = make_problem(32, 2, y=np.ones((32, 32)), sigma=0.1, max_batch=4)
    th = torch.tensor(np.array([THETA_TRUE] * 5), device="cuda")
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    st = torch.zeros(5, dtype=torch.int32, device="cuda")
    L = _lib.lib()
    assert L.log_likelihood_batch_noalloc(p.h, 5, _ptr(th), _ptr(out), _ptr(st), None,
                                          None) == _lib.RD_EINVAL          # n > max_batch
    assert L.log_likelihood_batch_noalloc(p.h, 4, _ptr(th), None, _ptr(st), None,
                                          None) == _lib.RD_EINVAL          # no phi
    p.close()
    p, _, _ = make_problem(256, 2, y=np.ones((256, 256)), sigma=0.1, max_batch=4)
    assert L.log_likelihood_batch_noalloc(p.h, 4, _ptr(th), _ptr(out), _ptr(st), None,
                                          None) == _lib.RD_EUNSUPPORTED    # cooperative tile
    p.close()
