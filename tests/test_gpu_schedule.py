"""GPU: the D2IP frame schedule (UPWS warm start, then frames with or
without TPP) through the C-ABI, against the FP64 oracle run the same way."""
import numpy as np
import pytest

from oracle import fit
from paper_2507_14046_amd import schedule
from tests.gpu_util import make_ctx, oracle_problem, problem, record, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("tpp", [True, False])
def test_schedule_with_warm_start_matches_oracle(lib, tpp):
    p = problem(16, 1, 2, 8, 21, frames=3, breathing=True)
    warm = problem(16, 1, 2, 8, 1021)  # same geometry, another phantom: the warm-start task
    ctx = make_ctx(lib, [p])
    ctx.set_adam(lr=1e-3)
    th_w = schedule.warm_start(ctx, p["theta0"], warm["dv"][0], 5)
    imgs, losses, _ = schedule.run_sequence(ctx, p["dv"], 6, 4, theta_start=th_w, tpp=tpp)
    ctx.close()
    pr = oracle_problem(p)
    # UPWS in the oracle: a one-frame fit of the warm measurement from theta0
    _, _, st = fit.fit_sequence(pr, p["theta0"].astype(np.float64),
                                [warm["dv"][0].astype(np.float64)], [5], 1e-3)
    dvs = [d.astype(np.float64) for d in p["dv"]]
    if tpp:
        ref, ref_losses, _ = fit.fit_sequence(pr, st.theta, dvs, [6, 4, 4], 1e-3)
        ref_losses = [l[-1] for l in ref_losses]
    else:
        ref, ref_losses = [], []
        for f, dv in enumerate(dvs):
            im, ls, _ = fit.fit_sequence(pr, st.theta, [dv], [6 if f == 0 else 4], 1e-3)
            ref.append(im[0])
            ref_losses.append(ls[0][-1])
    errs = [rel(imgs[f], ref[f]) for f in range(3)]
    lerr = [abs(losses[f] - ref_losses[f]) / ref_losses[f] for f in range(3)]
    record("schedule_upws", tpp=tpp, image_rel=errs, loss_rel=lerr)
    assert max(errs) < 1e-5, errs
    # after fitting, the residual p - dv is a small difference of nearly equal
    # vectors: the loss's relative error is the image-level error amplified
    # by |p| / |r|, hence the looser bound
    assert max(lerr) < 1e-4, lerr
