"""Per-kernel timing of a context (msm_profile_*): with msm_profile_only
only the named kernel is timed; without it every kernel of a call is."""
import pytest
import torch

from helpers import announce
from paper_0904_3151_amd import inputs as I

pytestmark = pytest.mark.gpu


def one_step(msm, ctx, Xd, Rd, w):
    S = msm.msm_project(ctx, Xd, Rd)
    P, m = msm.enumerate_pairs(ctx, S, w.ell, w.k, w.h)
    msm.msm_verify(ctx, Xd, P, w.metric, w.eps)
    torch.cuda.synchronize()


def test_profile_only_times_one_kernel(msm, ctx):
    w = I.TINY
    X, R = I.workload_inputs(w, sigma_mode="radius", n=5000)
    Xd, Rd = torch.from_numpy(X).cuda(), torch.from_numpy(R).cuda()
    announce("profile only")
    msm.msm_profile_reset(ctx)
    msm.msm_profile_only(ctx, "k_bucket")
    msm.msm_profile_enable(ctx, True)
    one_step(msm, ctx, Xd, Rd, w)
    msm.msm_profile_enable(ctx, False)
    got = msm.msm_profile_read(ctx)
    assert set(got) == {"k_bucket"} and got["k_bucket"][0] >= 1 and got["k_bucket"][1] > 0
    msm.msm_profile_reset(ctx)
    msm.msm_profile_only(ctx, None)
    msm.msm_profile_enable(ctx, True)
    one_step(msm, ctx, Xd, Rd, w)
    msm.msm_profile_enable(ctx, False)
    every = msm.msm_profile_read(ctx)
    assert "k_bucket" in every and {"k_verify", "k_verify_h"} & set(every)
    assert {"k_project_f32", "k_project_x3"} & set(every)
    msm.msm_profile_reset(ctx)
    with pytest.raises(msm.MSMError) as e:
        msm.msm_profile_only(ctx, "x" * 48)
    assert e.value.status == msm.MSM_E_INVALID
