"""The no-allocation operator apply (spp_apply_operator_noalloc) against
spp_apply_operator, through the C ABI: two calls in a row on one factor, the
second with fewer right-hand sides, each compared with the allocating entry
point on the same input.  Both run the same FFT kernels in the same order, so
the results agree to the operator parity bar (1e-12 relative; identical bits
are expected); a size beyond the 64 MiB scratch is rejected."""
import ctypes

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def field(nrhs, N, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N))


def test_noalloc_operator_matches_allocating_entry_point():
    from paper_1409_0297_amd import Solver, binding
    W = workloads.parity_2d()
    S = Solver(W.kind, W.n, W.d, W.b, W.coeff, omega=W.omega, tol=1e-10, max_iter=40)
    lib = binding.library()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    N = W.n * W.n
    for nrhs, seed in ((6, 101), (2, 102)):
        z = torch.as_tensor(field(nrhs, N, seed), dtype=torch.complex128, device="cuda").contiguous()
        w_ref = torch.empty_like(z)
        w_new = torch.full_like(z, float("nan"))
        assert lib.spp_apply_operator(S.handle, z.data_ptr(), w_ref.data_ptr(), nrhs, stream) == 0
        assert lib.spp_apply_operator_noalloc(S.handle, z.data_ptr(), w_new.data_ptr(), nrhs, stream) == 0
        torch.cuda.synchronize()
        a, b = w_new.cpu().numpy(), w_ref.cpu().numpy()
        assert np.all(np.isfinite(a))
        e = np.linalg.norm(a - b) / np.linalg.norm(b)
        assert e <= 1e-12, (nrhs, e)
    # nrhs * N * 16 bytes beyond the 64 MiB scratch: rejected before any launch
    big = (64 << 20) // (16 * N) + 1
    assert lib.spp_apply_operator_noalloc(S.handle, z.data_ptr(), w_new.data_ptr(), big, stream) == -1
    S.close()
