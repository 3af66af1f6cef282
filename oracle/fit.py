"""FP64 oracle of the D2IP fitting iteration, Adam and the frame schedule.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

One iteration for frame i (Eqs. (3)-(4), Adam on theta as in Sec. III-A):

  1. image  d_sigma = mask * phi(theta | Z)               (Eq. (3), reshaped by V)
  2. predicted voltages p = J d_sigma                      (Eq. (1))
  3. residual r = p - dv_i; data loss L = (1/M) sum r^2    (the l2 data term of
     Eq. (4), in the mean-squared form the paper calls its "MSE loss", Sec. V-A)
  4. dL/d(d_sigma) = (2/M) J^T r, masked
  5. dL/dtheta by reverse-mode through the network
  6. Adam step (Kingma & Ba): t += 1; m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2;
     theta -= lr * (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps)

The loss recorded for an iteration is evaluated at the parameters before its
update.  After N_i iterations the frame's image is mask * phi(theta^(N_i) | Z)
(Eq. (5)).  Frame i+1 starts from theta^(N_i) of frame i (TPP, Eq. (9)); by
default the Adam moments and step counter restart at zero on every frame,
since the paper transfers only theta.
"""
import numpy as np

from . import net
from . import tv as tvmod

ADAM_BETA1 = 0.9
ADAM_BETA2 = 0.999
ADAM_EPS = 1e-8


def data_loss(J, dv, sigma):
    """(L, dL/dsigma) for L = (1/M) ||J sigma - dv||^2."""
    M = J.shape[0]
    r = J @ sigma - dv
    return float(r @ r) / M, (2.0 / M) * (J.T @ r)


def adam_step(theta, g, m, v, t, lr, b1=ADAM_BETA1, b2=ADAM_BETA2, eps=ADAM_EPS):
    """One Adam update; returns (theta, m, v, t) as new arrays."""
    t = t + 1
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** t)
    vhat = v / (1.0 - b2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v, t


class Problem:
    """Inputs of one instance promoted to FP64."""

    def __init__(self, J, mask, Z, n, levels, base_ch, sep=False, se_ratio=0, att=False,
                 tail="linear", aspp=False):
        self.J = np.asarray(J, dtype=np.float64)
        self.mask = np.asarray(mask, dtype=np.float64)
        self.Z = np.asarray(Z, dtype=np.float64)
        self.n, self.levels, self.base_ch = n, levels, base_ch
        self.sep = sep  # depthwise-separable ResBlock convolutions
        self.se_ratio = se_ratio  # SE units after the encoder blocks (0: none)
        self.att, self.tail = att, tail  # attention units on the skips; output head
        self.aspp = aspp  # ASPP module at the bottleneck

    def image(self, theta):
        out, _ = net.forward(theta, self.Z, self.n, self.levels, self.base_ch, self.sep,
                                 self.se_ratio, self.att, self.tail, self.aspp)
        return self.mask * out.ravel()

    def loss_and_grad(self, theta, dv, tv=None):
        """(L, dL/dtheta, image) at theta for one frame: the data term, plus
        the 4D-TV term when tv = dict(history=[images], weights=[...],
        lam=, lam_s=, lam_t=, eps=) is given (Eq. (14))."""
        out, cache = net.forward(theta, self.Z, self.n, self.levels, self.base_ch, self.sep,
                                 self.se_ratio, self.att, self.tail, self.aspp)
        sigma = self.mask * out.ravel()
        L, gs = data_loss(self.J, dv, sigma)
        if tv is not None:
            n = self.n
            hist = [np.asarray(h, dtype=np.float64).reshape(n, n, n) for h in tv["history"]]
            Lt, gt = tvmod.tv4d(sigma.reshape(n, n, n), hist, tv["weights"], tv["lam"],
                                tv["lam_s"], tv["lam_t"], tv["eps"])
            L += Lt
            gs = gs + gt.ravel()
        gout = (self.mask * gs).reshape(self.n, self.n, self.n)
        g = net.backward(gout, theta, cache, self.n, self.levels, self.base_ch, self.sep,
                         self.se_ratio, self.att, self.tail, self.aspp)
        return L, g, sigma


class State:
    """theta and the Adam state of one instance."""

    def __init__(self, theta):
        self.theta = np.asarray(theta, dtype=np.float64).copy()
        self.m = np.zeros_like(self.theta)
        self.v = np.zeros_like(self.theta)
        self.t = 0

    def reset_optimizer(self):
        self.m[...] = 0.0
        self.v[...] = 0.0
        self.t = 0


def run(problem, state, dv, k, lr, b1=ADAM_BETA1, b2=ADAM_BETA2, eps=ADAM_EPS, tv=None):
    """k Adam iterations on one frame; returns the k recorded losses."""
    dv = np.asarray(dv, dtype=np.float64)
    losses = []
    for _ in range(k):
        L, g, _ = problem.loss_and_grad(state.theta, dv, tv)
        state.theta, state.m, state.v, state.t = adam_step(
            state.theta, g, state.m, state.v, state.t, lr, b1, b2, eps)
        losses.append(L)
    return losses


def fit_sequence(problem, theta0, dvs, iters, lr, reset_on_frame=True,
                 b1=ADAM_BETA1, b2=ADAM_BETA2, eps=ADAM_EPS, tv=None):
    """Frames in order with TPP.  iters[i] = N_i.  Returns (images, losses).

    With tv = dict(lam=, lam_s=, lam_t=, eps=) every frame's loss carries the
    4D-TV term, its temporal part over all earlier frames' final images."""
    st = State(theta0)
    images, losses = [], []
    for i, dv in enumerate(dvs):
        if reset_on_frame:
            st.reset_optimizer()
        frame_tv = None
        if tv is not None:
            frame = i + 1  # 1-based frame index of Eq. (13)
            prev = list(range(1, frame))
            frame_tv = dict(tv, history=list(images),
                            weights=tvmod.temporal_weights(frame, prev) if prev else [])
        losses.append(run(problem, st, dv, iters[i], lr, b1, b2, eps, frame_tv))
        images.append(problem.image(st.theta))
    return np.stack(images), losses, st
