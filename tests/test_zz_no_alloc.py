"""The allocation-free entry point (nmf_closest_frames_noalloc), through the
C ABI, against the allocating one (nmf_closest_frames) on the same inputs:
bit-exact indices (the same kernels run on the same data), on two calls in a
row, the second with a smaller input (the scratch array keeps the first
call's contents), plus the host-side capacity check."""
import numpy as np
import pytest

from paper_2309_04623_amd import nmf
from tests.helpers import dev, say

pytestmark = pytest.mark.gpu


def _case(seed, f, n, p):
    g = np.random.default_rng(seed)
    V = g.gamma(2, 1, (n, p)).astype(np.float32)
    T = g.gamma(2, 1, (f, p)).astype(np.float32)
    M = (g.random((n, p)) > 0.05).astype(np.float32)
    MT = (g.random((f, p)) > 0.05).astype(np.float32)
    V[M == 0] = np.nan
    return dev(V), dev(M), dev(T), dev(MT)


def test_noalloc_matches_allocating_entry_point_on_two_calls():
    h = nmf.Handle(0)
    for seed, f, n, p, n_sel in ((1, 6, 500, 4000, 40), (2, 3, 200, 1500, 17)):
        V, M, T, MT = _case(seed, f, n, p)
        say("noalloc closest frames", f, n, p, n_sel)
        ref = nmf.closest_frames(V, M, T, MT, n_sel, handle=h)
        got = nmf.closest_frames_noalloc(V, M, T, MT, n_sel, handle=h)
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())


def test_noalloc_rejects_requests_beyond_the_scratch():
    V, M, T, MT = _case(3, 2, 40, 64)
    say("noalloc capacity")
    big_f, big_n = 64, 40000  # 2.56e6 distances > 2,097,120
    with pytest.raises(nmf.NmfError) as e:
        nmf.lib()
        import ctypes
        st = nmf.lib().nmf_closest_frames_noalloc(
            nmf.default_handle(0).h, V.data_ptr(), M.data_ptr(), big_n, 64, T.data_ptr(),
            MT.data_ptr(), big_f, 1, V.data_ptr(), None)
        nmf._check(st)
    assert e.value.status == nmf.NMF_ERR_UNSUPPORTED
