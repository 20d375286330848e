"""Batched nested sampling on the batched likelihood (paper Sec. 2.5).

The paper estimates the evidence Z and posterior with nested sampling: N live
points drawn from the prior; the worst one is replaced by a new prior draw
with a higher likelihood; the enclosed prior mass shrinks as X_t = t X_{t-1}
with t the largest of N uniforms; Z accumulates L (X_{t-1} - X_t) until the
remaining contribution would change it by less than a fraction f.  Two models
are compared through the ratio of their evidences (the Bayes factor; the
odds ratio with equal model priors).

Here each iteration removes the k worst live points at once (in likelihood
order, the live count falling from N to N - k + 1, so the i-th removal
shrinks log X by 1 / (N - i + 1) in expectation) and replaces them with k new
points, each found by a constrained random walk started from a surviving live
point, all k walks advancing together so that every step is one batched
likelihood call.  The bookkeeping of an iteration (sort, shrinkage, evidence
update, stopping test) is a fixed sequence of tensor operations on the
device, so with ``graph=True`` one whole iteration, walk steps included, is
captured once in a HIP graph and replayed; the host reads the stopping flag
only every ``check_every`` iterations (iterations past the stopping point are
ordinary nested-sampling iterations and leave the estimate valid).

Works with any batched log-likelihood: a callable taking a [B, P] float64
tensor (in the sampling coordinates) and returning [B] logL, such as
``Grid.loglike`` or ``LogLike``; for ``graph=True`` it must enqueue its work
on the current stream and allocate only through torch (``Grid.loglike``
does).  The prior is uniform on a box.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable, List, Optional

import torch


@dataclass
class NestedResult:
    log_z: float                 # log evidence
    log_z_err: float             # sqrt(H / N), the usual statistical error
    information: float           # H, nats
    n_iter: int
    n_like: int                  # likelihood evaluations
    samples: torch.Tensor        # dead points, [M, P]
    log_w: torch.Tensor          # their log posterior weights (normalised)
    log_l: torch.Tensor          # their log-likelihoods
    history: List[float] = field(default_factory=list)

    def posterior_mean(self) -> torch.Tensor:
        w = torch.exp(self.log_w - self.log_w.max())
        return (w[:, None] * self.samples).sum(0) / w.sum()


def log_bayes_factor(a: NestedResult, b: NestedResult):
    """ln(Z_a / Z_b) and its statistical error (the two runs' errors in
    quadrature): the log odds ratio of model a over model b for equal model
    priors (Sec. 2.5)."""
    return a.log_z - b.log_z, math.hypot(a.log_z_err, b.log_z_err)


class _State:
    """Device tensors of one run; every iteration updates them in place."""

    def __init__(self, loglike, lo, hi, n_live, k, f, walk_steps, gen):
        self.loglike, self.lo, self.hi, self.k, self.walk_steps, self.gen = loglike, lo, hi, k, walk_steps, gen
        dev, P = lo.device, lo.numel()
        self.width = hi - lo
        self.scale_floor = 1e-12 * float(self.width.max())     # host value: no sync inside a capture
        self.live = lo + self.width * torch.rand(n_live, P, dtype=torch.float64, device=dev, generator=gen)
        self.live_l = loglike(self.live).to(torch.float64).clone()
        self.log_x = torch.zeros((), dtype=torch.float64, device=dev)
        self.log_z = torch.full((), -math.inf, dtype=torch.float64, device=dev)
        self.stop = torch.zeros((), dtype=torch.bool, device=dev)
        self.log_f = math.log(f)
        # the k removals of an iteration, live count N .. N - k + 1: shrinkage of
        # log X by -1/n_i each (constants of the run)
        n_i = n_live - torch.arange(k, dtype=torch.float64, device=dev)
        self.dlog = -1.0 / n_i
        self.cum = torch.cumsum(self.dlog, 0)
        self.log_frac = torch.log(-torch.expm1(self.dlog))      # log(1 - X_i / X_{i-1})
        # what each iteration hands back: the removed points and their weights
        self.dead_x = torch.empty(k, P, dtype=torch.float64, device=dev)
        self.dead_l = torch.empty(k, dtype=torch.float64, device=dev)
        self.dead_lw = torch.empty(k, dtype=torch.float64, device=dev)

    def iteration(self):
        k, live, live_l = self.k, self.live, self.live_l
        order = torch.argsort(live_l)
        worst, keep = order[:k], order[k:]
        wl = live_l[worst]
        # removals in likelihood order: X_{i-1} = X exp(cum_i - dlog_i)
        lw = wl + self.log_x + (self.cum - self.dlog) + self.log_frac
        self.log_z.copy_(torch.logaddexp(self.log_z, torch.logsumexp(lw, 0)))
        self.log_x.add_(self.cum[-1])
        self.dead_x.copy_(live[worst])
        self.dead_l.copy_(wl)
        self.dead_lw.copy_(lw)
        # replacements: constrained random walks from surviving live points
        l_min = wl[-1]
        start = keep[torch.randint(0, keep.numel(), (k,), device=live.device, generator=self.gen)]
        x = live[start]
        xl = live_l[start]
        # proposal: a fraction of the surviving live points' spread per axis
        scale = live[keep].std(0).clamp_min(self.scale_floor) * 0.5
        for _ in range(self.walk_steps):
            prop = x + scale * torch.randn(k, live.shape[1], dtype=torch.float64, device=live.device,
                                           generator=self.gen)
            inside = ((prop >= self.lo) & (prop <= self.hi)).all(1)
            prop_eval = torch.where(inside[:, None], prop, x)
            pl = self.loglike(prop_eval).to(torch.float64)
            ok = inside & (pl > l_min)
            x = torch.where(ok[:, None], prop, x)
            xl = torch.where(ok, pl, xl)
        live[worst] = x
        live_l[worst] = xl
        # stop: the live points can add at most max(L) X to Z
        self.stop.copy_(live_l.max() + self.log_x < self.log_z + self.log_f)


def nested_sampling(loglike: Callable[[torch.Tensor], torch.Tensor], lo, hi, n_live: int = 400,
                    k: Optional[int] = None, f: float = 1e-3, walk_steps: int = 25,
                    max_iter: int = 100000, generator: Optional[torch.Generator] = None,
                    device=None, graph: bool = False, check_every: int = 1) -> NestedResult:
    """Evidence and posterior samples for a uniform prior on the box [lo, hi].

    n_live: N live points; k: points replaced per iteration (default N/10);
    f: stop when the live points can add less than a fraction f to Z;
    walk_steps: constrained random-walk steps per new point; graph: capture
    one iteration in a HIP graph and replay it (GPU only); check_every: read
    the stopping flag on the host every this many iterations."""
    lo = torch.as_tensor(lo, dtype=torch.float64, device=device)
    hi = torch.as_tensor(hi, dtype=torch.float64, device=device)
    dev = lo.device
    k = k or max(1, n_live // 10)
    if not 1 <= k < n_live:
        raise ValueError("need 1 <= k < n_live")
    if graph and dev.type != "cuda":
        raise ValueError("graph=True needs a GPU device")
    st = _State(loglike, lo, hi, n_live, k, f, walk_steps, generator)
    dead, dead_l, dead_lw = [], [], []
    history: List[torch.Tensor] = []

    def collect():
        dead.append(st.dead_x.clone())
        dead_l.append(st.dead_l.clone())
        dead_lw.append(st.dead_lw.clone())
        history.append(st.log_z.clone())

    step = st.iteration
    if graph:
        # the first iteration runs eagerly on a side stream (loads the kernels
        # and lets the allocator settle), then one iteration is captured
        side = torch.cuda.Stream(device=dev)
        side.wait_stream(torch.cuda.current_stream(dev))
        with torch.cuda.stream(side):
            st.iteration()
        torch.cuda.current_stream(dev).wait_stream(side)
        collect()
        g = torch.cuda.CUDAGraph()
        if generator is not None:
            g.register_generator_state(generator)
        with torch.cuda.graph(g):
            st.iteration()
        step = g.replay
        it = 1
    else:
        it = 0
    stopped = it > 0 and bool(st.stop)
    while not stopped and it < max_iter:
        step()
        it += 1
        collect()
        if it % check_every == 0 or it == max_iter:
            stopped = bool(st.stop)
    # the remaining live points share the final X equally
    lw_live = st.live_l + (st.log_x - math.log(n_live))
    log_z_t = torch.logaddexp(st.log_z, torch.logsumexp(lw_live, 0))
    samples = torch.cat(dead + [st.live.clone()])
    log_l = torch.cat(dead_l + [st.live_l.clone()])
    log_w = torch.cat(dead_lw + [lw_live]) - log_z_t
    log_z = float(log_z_t)
    w = torch.exp(log_w)
    info = max(float((w * (log_l - log_z)).sum()), 0.0)
    hist = torch.stack(history).tolist() if history else []
    return NestedResult(log_z=log_z, log_z_err=math.sqrt(info / n_live), information=info,
                        n_iter=it, n_like=n_live + it * k * walk_steps, samples=samples, log_w=log_w,
                        log_l=log_l, history=hist)
