"""unweight_noalloc (fixed device scratch, no allocation) against unweight
(stream-ordered scratch): the same kept indices, count and bound, bit for
bit, on consecutive calls of decreasing size (the array keeps the previous
call's contents), with the bound searched and given."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def weights(n, seed):
    import torch
    g = torch.Generator(device="cuda").manual_seed(seed)
    # a steep spectrum: efficiency of a few per cent, as for event weights
    u = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
    return u ** 12


def both(vgx, w, seed, sid, it, w_max=0.0):
    import torch
    n = w.numel()
    i1 = torch.full((n,), -1, dtype=torch.int64, device="cuda")
    i2 = torch.full((n,), -2, dtype=torch.int64, device="cuda")
    k1, m1 = vgx.unweight(w, seed, sid, it, i1, w_max=w_max)
    k2, m2 = vgx.unweight_noalloc(w, seed, sid, it, i2, w_max=w_max)
    torch.cuda.synchronize()
    return (k1, m1, i1[:k1].cpu().numpy()), (k2, m2, i2[:k2].cpu().numpy())


@pytest.mark.parametrize("n1,n2", [(3_000_017, 123_457), (65_536, 4_095)])
def test_noalloc_matches_unweight_on_consecutive_calls(vgx, n1, n2):
    print(f"unweight_noalloc vs unweight: n = {n1} then {n2}", flush=True)
    for n, seed, w_max in ((n1, 5, 0.0), (n2, 6, 0.0), (n2, 7, 0.5)):
        w = weights(n, seed)
        (k1, m1, a1), (k2, m2, a2) = both(vgx, w, 21, 3, seed, w_max)
        print(f"  n {n}: kept {k1} / {k2}, bound {m1:.6g} / {m2:.6g}", flush=True)
        assert k1 == k2 and k1 > 0
        assert m1 == m2
        assert np.array_equal(a1, a2)
        assert np.all(np.diff(a2) > 0) and a2[0] >= 0 and a2[-1] < n


def test_noalloc_rejects_more_than_its_scratch_holds(vgx):
    """Beyond the fixed array: VGX_EINVAL from the host-side size check,
    before anything is launched (the buffers passed are never touched)."""
    import torch
    w = torch.ones(16, dtype=torch.float64, device="cuda")
    idx = torch.empty(16, dtype=torch.int64, device="cuda")
    k, wm = C.c_int64(), C.c_double()
    st = vgx._c["unweight_noalloc"](vgx.UNWEIGHT_NOALLOC_MAX + 1, C.c_void_p(w.data_ptr()), 0.0, 1, 0, 0,
                                    C.c_void_p(idx.data_ptr()), C.byref(k), C.byref(wm), None)
    assert st == vgx.VGX_EINVAL
    assert "scratch" in vgx.last_error()
    # the largest accepted size is the documented one
    assert vgx.UNWEIGHT_NOALLOC_MAX == 16100 * 4096
