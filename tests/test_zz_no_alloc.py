"""msm_enumerate_pairs_noalloc (the entry point for callers that cannot
allocate) against msm_enumerate_pairs: the same pair set, bit for bit, on two
calls in a row, the second with a smaller input of another shape, and a
clear rejection of an input whose work memory exceeds the fixed buffer."""
import ctypes

import numpy as np
import pytest
import torch

from helpers import announce, codes, to_np_pairs
from paper_0904_3151_amd import inputs as I

pytestmark = pytest.mark.gpu


def strings_of(msm, ctx, w, n, sigma_mode):
    X, R = I.workload_inputs(w, sigma_mode=sigma_mode, n=n)
    return msm.msm_project(ctx, torch.from_numpy(X).cuda(), torch.from_numpy(R).cuda())


def raw_noalloc(msm, ctx, S, ell, k, h, pairs):
    """The C entry point itself, through ctypes."""
    m = ctypes.c_int64(-1)
    st = msm.lib().msm_enumerate_pairs_noalloc(ctx.handle, ctypes.c_void_p(S.data_ptr()), S.shape[0], ell, k, h,
                                               ctypes.c_void_p(pairs.data_ptr()), pairs.shape[0], ctypes.byref(m),
                                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    return st, m.value


@pytest.mark.parametrize("first,second", [
    # paper-scale shape on 120k points (8 partition tiles, hierarchical
    # grouping), then the tiny shape on 9k points
    ((I.PAPER_SCALE, 120_000, "radius"), (I.TINY, 9_000, "radius")),
    ((I.PAPER_SCALE, 60_000, "coord"), (I.PAPER_SCALE, 5_000, "coord")),
])
def test_noalloc_matches_enumerate(msm, ctx, first, second):
    for w, n, mode in (first, second):
        announce("noalloc", w.name, n, mode)
        S = strings_of(msm, ctx, w, n, mode)
        want, m_want = msm.enumerate_pairs(ctx, S, w.ell, w.k, w.h)
        pairs = torch.full((m_want + 1000, 2), -1, dtype=torch.int32, device="cuda")
        st, m = raw_noalloc(msm, ctx, S, w.ell, w.k, w.h, pairs)
        assert st == msm.MSM_OK, ctx.last_error()
        assert m == m_want
        got = codes(to_np_pairs(pairs[:m]))
        assert np.array_equal(got, codes(to_np_pairs(want)))
        assert np.all(got[1:] != got[:-1])


def test_noalloc_capacity_and_count_only(msm, ctx):
    w = I.TINY
    S = strings_of(msm, ctx, w, 20_000, "radius")
    _, m_want = msm.enumerate_pairs(ctx, S, w.ell, w.k, w.h)
    announce("noalloc count only", m_want)
    _, m = msm.msm_enumerate_pairs_noalloc(ctx, S, w.ell, w.k, w.h, cap=0)
    assert m == m_want
    small = torch.empty((max(1, m_want // 2), 2), dtype=torch.int32, device="cuda")
    with pytest.raises(msm.MSMError) as e:
        msm.msm_enumerate_pairs_noalloc(ctx, S, w.ell, w.k, w.h, pairs=small)
    assert e.value.status == msm.MSM_E_CAPACITY and e.value.required == m_want


def test_noalloc_rejects_inputs_beyond_the_buffer(msm, ctx):
    # 8M random strings need about 75 MB of work memory, above the 64 MiB
    # buffer: rejected before any work
    n = 8_000_000
    S = torch.randint(-(1 << 62), 1 << 62, (n, 2), dtype=torch.int64, device="cuda")
    pairs = torch.empty((16, 2), dtype=torch.int32, device="cuda")
    announce("noalloc too large", n)
    st, m = raw_noalloc(msm, ctx, S, 128, 8, 4, pairs)
    assert st == msm.MSM_E_UNSUPPORTED
    assert m == 0
    assert "no-allocation buffer" in ctx.last_error()
    # the regular entry point takes the same input (a count only)
    _, m_reg = msm.msm_enumerate_pairs(ctx, S, 128, 8, 4, cap=0)
    assert m_reg >= 0
