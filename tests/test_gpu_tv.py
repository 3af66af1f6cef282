"""GPU parity of the 4D-TV term (Sec. III-E, Eqs. (11)-(14)) against the FP64
oracle: the loss and gradient of an iteration with a two-frame history, and a
three-frame sequence fitted with TPP and the regulariser."""
import numpy as np
import pytest

from oracle import fit, tv
from tests.gpu_util import make_ctx, oracle_problem, problem, record, rel

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("lam", [0.002, 0.05])
def test_tv_iteration_gradient_with_history(lib, lam):
    p = problem(16, 1, 2, 8, 61, frames=3, breathing=True)
    ctx = make_ctx(lib, [p])
    ctx.set_tv(lambda_tv=lam, lambda_s=1.0, lambda_t=0.1, eps=1e-8)
    ctx.run(2)
    ctx.commit_frame(0)
    ctx.set_frame(0, p["dv"][1])
    ctx.reset_optimizer(0)
    ctx.run(2)
    ctx.commit_frame(0)
    ctx.set_frame(0, p["dv"][2])
    ctx.reset_optimizer(0)
    loss = ctx.run(1)[0]
    g = ctx.get_grad(0)
    pr = oracle_problem(p)
    cfg = dict(lam=lam, lam_s=1.0, lam_t=0.1, eps=1e-8)
    imgs, _, st = fit.fit_sequence(pr, p["theta0"], p["dv"][:2], [2, 2], 1e-3, tv=cfg)
    L, gref, _ = pr.loss_and_grad(st.theta, p["dv"][2].astype(np.float64),
                                  dict(cfg, history=list(imgs),
                                       weights=tv.temporal_weights(3, [1, 2])))
    e = dict(loss=abs(loss - L) / L, grad=rel(g, gref))
    record("tv_iteration", lam=lam, **e)
    assert e["loss"] < 1e-5 and e["grad"] < 2e-4, e


@pytest.mark.parametrize("graph", [False, True])
def test_tv_sequence_matches_oracle(lib, graph):
    p = problem(16, 1, 2, 8, 62, frames=3, breathing=True)
    ctx = make_ctx(lib, [p], graph=graph)
    ctx.set_tv()
    iters = [6, 4, 4]
    imgs = []
    for f in range(3):
        if f:
            ctx.commit_frame(0)
            ctx.set_frame(0, p["dv"][f])
            ctx.reset_optimizer(0)
        ctx.run(iters[f])
        imgs.append(ctx.read_image(0))
    pr = oracle_problem(p)
    ref, _, _ = fit.fit_sequence(pr, p["theta0"], p["dv"], iters, 1e-3,
                                 tv=dict(lam=0.002, lam_s=1.0, lam_t=0.1, eps=1e-8))
    e = [rel(imgs[f], ref[f]) for f in range(3)]
    record("tv_sequence", graph=graph, image_rel=e)
    assert max(e) < 1e-5, e
