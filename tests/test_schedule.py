"""Host logic of the D2IP frame schedule (UPWS, TPP, iterations to a target
loss, the ablation's bookkeeping) against a scalar stand-in for a context
whose iteration is plain gradient descent on (theta - dv)^2, simulated here
independently."""
import numpy as np
import pytest

from paper_2507_14046_amd import schedule as sch

STEP = 0.1


class FakeCtx:
    """One instance; theta is a 1-vector; run(k) does k gradient steps
    theta += STEP * (dv - theta) and reports the loss before the last one."""

    def __init__(self, theta0):
        self.instances = [(0, 3, 16)]
        self.theta = np.array(theta0, dtype=np.float64)
        self.dv = 0.0
        self.runs = []
        self.history = []
        self.lr = None

    def set_adam(self, lr):
        self.lr = lr

    def set_params(self, inst, theta):
        self.theta = np.array(theta, dtype=np.float64)

    def get_params(self, inst):
        return self.theta.copy()

    def set_frame(self, inst, dv):
        self.dv = float(dv)

    def reset_optimizer(self, inst):
        pass

    def clear_history(self, inst):
        self.history = []

    def commit_frame(self, inst):
        self.history.append(float(self.theta[0]))

    def read_image(self, inst):
        return self.theta.copy()

    def run(self, k, sync=True):
        self.runs.append(k)
        loss = None
        for _ in range(k):
            loss = (self.theta[0] - self.dv) ** 2
            self.theta[0] += STEP * (self.dv - self.theta[0])
        return np.array([loss])


def gd(theta, dv, k):
    """theta after k steps and the loss before the last one (closed form)."""
    r = (theta - dv) * (1 - STEP) ** np.arange(k + 1)
    return dv + r[k], r[k - 1] ** 2


def test_warm_start_fits_the_warm_frame_from_theta0():
    ctx = FakeCtx([5.0])
    th = sch.warm_start(ctx, [2.0], 7.0, 30)
    assert th[0] == pytest.approx(gd(2.0, 7.0, 30)[0], rel=1e-12)
    assert sch.warm_start(ctx, [2.0], 7.0, 0)[0] == 2.0


@pytest.mark.parametrize("tpp", [True, False])
def test_run_sequence_carries_or_restarts_parameters(tpp):
    ctx = FakeCtx([1.0])
    dvs = [4.0, -2.0, 3.0]
    imgs, losses, secs = sch.run_sequence(ctx, dvs, 12, 5, theta_start=[0.5], tpp=tpp, tv=True)
    th, want_imgs, want_losses = 0.5, [], []
    for f, dv in enumerate(dvs):
        start = th if tpp else 0.5
        th, loss = gd(start, dv, 12 if f == 0 else 5)
        want_imgs.append(th)
        want_losses.append(loss)
    np.testing.assert_allclose(imgs[:, 0], want_imgs, rtol=1e-12)
    np.testing.assert_allclose(losses, want_losses, rtol=1e-12)
    assert ctx.history == pytest.approx(want_imgs, rel=1e-12)  # every frame committed
    assert ctx.runs == [12, 5, 5] and secs >= 0


@pytest.mark.parametrize("target,cap,chunk", [(1.0, 100, 10), (1e-3, 100, 7), (1e-30, 25, 10)])
def test_iterations_to_target_stops_at_the_first_chunk_below(target, cap, chunk):
    ctx = FakeCtx([0.0])
    ctx.set_frame(0, 3.0)
    k, loss, ok = sch.iterations_to_target(ctx, target, cap, chunk)
    # brute force: chunk boundaries until the loss before the last step <= target
    want_k, want_ok = None, False
    b = 0
    while b < cap:
        b = min(b + chunk, cap)
        if gd(0.0, 3.0, b)[1] <= target:
            want_k, want_ok = b, True
            break
    if want_k is None:
        want_k = cap
    assert (k, ok) == (want_k, want_ok)
    assert loss == pytest.approx(gd(0.0, 3.0, k)[1], rel=1e-12)


def test_ablation_bookkeeping():
    theta0, dv_warm, dvs = [0.0], 5.0, [5.5, 6.0, 6.5]
    sched = dict(upws=40, first=20, later=10, lr=5e-4)
    ctx = FakeCtx(theta0)
    res = sch.ablation(ctx, theta0, dvs, dv_warm, sched=sched, target_factor=1.05,
                       cap_factor=8, chunk=5)
    assert ctx.lr == 5e-4
    # the full schedule and its per-frame targets, simulated here
    th_w = gd(0.0, dv_warm, 40)[0]
    th, finals = th_w, []
    for f, dv in enumerate(dvs):
        th, loss = gd(th, dv, 20 if f == 0 else 10)
        finals.append(loss)
    np.testing.assert_allclose(res["scheduled_full"]["final_losses"], finals, rtol=1e-12)
    assert res["scheduled_full"]["iterations"] == 40
    targets = 1.05 * np.array(finals)

    def variant(start, tpp):
        th, its = start, []
        for f, dv in enumerate(dvs):
            s = th if tpp else start
            cap = 8 * (20 if f == 0 else 10)
            k = 0
            while k < cap:
                k = min(k + 5, cap)
                if gd(s, dv, k)[1] <= targets[f]:
                    break
            its.append(k)
            th = gd(s, dv, k)[0]
        return its

    for name, upws, tpp in sch.VARIANTS:
        v = res["variants"][name]
        assert v["iterations"] == variant(th_w if upws else 0.0, tpp), name
        assert v["total_iterations"] == sum(v["iterations"])
    full = res["variants"]["full"]
    assert full["all_reached"] and full["iterations_vs_full"] == 1.0
    # the warm start and propagation pay off on this problem
    assert res["variants"]["no_upws_no_tpp"]["total_iterations"] > full["total_iterations"]


def test_schedule_rejects_multi_instance_contexts():
    ctx = FakeCtx([0.0])
    ctx.instances = [(0, 3, 16), (0, 3, 16)]
    with pytest.raises(ValueError):
        sch.run_sequence(ctx, [1.0], 1, 1)
