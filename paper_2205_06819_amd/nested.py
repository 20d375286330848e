"""Batched nested sampling on the batched likelihood (paper Sec. 2.5).

The paper estimates the evidence Z and posterior with nested sampling: N live
points drawn from the prior; the worst one is replaced by a new prior draw
with a higher likelihood; the enclosed prior mass shrinks as X_t = t X_{t-1}
with t the largest of N uniforms; Z accumulates L (X_{t-1} - X_t) until the
remaining contribution would change it by less than a fraction f.

Here each iteration removes the k worst live points at once (in likelihood
order, the live count falling from N to N - k + 1, so the i-th removal
shrinks log X by 1 / (N - i + 1) in expectation) and replaces them with k new
points, each found by a constrained random walk started from a surviving live
point, all k walks advancing together so that every step is one batched
likelihood call.  Works with any batched log-likelihood: a callable taking a
[B, P] float64 tensor (in the sampling coordinates) and returning [B] logL,
such as ``Grid.loglike`` or ``LogLike``.  The prior is uniform on a box.
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


def _logaddexp(a: float, b: float) -> float:
    if a == -math.inf:
        return b
    if b == -math.inf:
        return a
    m = max(a, b)
    return m + math.log(math.exp(a - m) + math.exp(b - m))


def nested_sampling(loglike: Callable[[torch.Tensor], torch.Tensor], lo, hi, n_live: int = 400,
                    k: Optional[int] = None, f: float = 1e-3, walk_steps: int = 25,
                    max_iter: int = 100000, generator: Optional[torch.Generator] = None,
                    device=None) -> NestedResult:
    """Evidence and posterior samples for a uniform prior on the box [lo, hi].

    n_live: N live points; k: points replaced per iteration (default N/10);
    f: stop when the live points can add less than a fraction f to Z;
    walk_steps: constrained random-walk steps per new point."""
    lo = torch.as_tensor(lo, dtype=torch.float64, device=device)
    hi = torch.as_tensor(hi, dtype=torch.float64, device=device)
    dev = lo.device
    P = lo.numel()
    k = k or max(1, n_live // 10)
    if not 1 <= k < n_live:
        raise ValueError("need 1 <= k < n_live")
    g = generator
    width = hi - lo

    def prior_draw(n):
        return lo + width * torch.rand(n, P, dtype=torch.float64, device=dev, generator=g)

    live = prior_draw(n_live)
    live_l = loglike(live).to(torch.float64)
    n_like = n_live
    log_z = -math.inf
    log_x = 0.0
    dead, dead_l, dead_lw = [], [], []
    history = []
    it = 0
    while it < max_iter:
        it += 1
        order = torch.argsort(live_l)
        worst = order[:k]
        wl = live_l[worst]
        wl_host = wl.tolist()            # one device-to-host copy per iteration
        # the k removals in likelihood order: the i-th shrinks X by ~1/(N - i + 1)
        for i in range(k):
            n_i = n_live - i
            log_x_new = log_x - 1.0 / n_i
            log_dx = log_x + math.log(-math.expm1(log_x_new - log_x))
            lw = wl_host[i] + log_dx
            log_z = _logaddexp(log_z, lw)
            log_x = log_x_new
            dead_lw.append(lw)
        dead.append(live[worst].clone())
        dead_l.append(wl.clone())
        # replacements: constrained random walks from surviving live points
        l_min = wl_host[-1]
        keep = order[k:]
        start = keep[torch.randint(0, keep.numel(), (k,), device=dev, generator=g)]
        x = live[start].clone()
        xl = live_l[start].clone()
        # proposal: a fraction of the surviving live points' spread per axis
        scale = live[keep].std(0).clamp_min(1e-12 * float(width.max())) * 0.5
        for _ in range(walk_steps):
            prop = x + scale * torch.randn(k, P, dtype=torch.float64, device=dev, generator=g)
            inside = ((prop >= lo) & (prop <= hi)).all(1)
            prop_eval = torch.where(inside[:, None], prop, x)
            pl = loglike(prop_eval).to(torch.float64)
            n_like += k
            ok = inside & (pl > l_min)
            x = torch.where(ok[:, None], prop, x)
            xl = torch.where(ok, pl, xl)
        live[worst] = x
        live_l[worst] = xl
        history.append(log_z)
        # stop: the live points can add at most max(L) X to Z
        l_max = float(live_l.max())
        if l_max + log_x < log_z + math.log(f):
            break
    # the remaining live points share the final X equally
    lx = log_x - math.log(n_live)
    for li in live_l.tolist():
        lw = li + lx
        log_z = _logaddexp(log_z, lw)
        dead_lw.append(lw)
    dead.append(live.clone())
    dead_l.append(live_l.clone())
    samples = torch.cat(dead)
    log_l = torch.cat(dead_l)
    log_w = torch.tensor(dead_lw, dtype=torch.float64, device=dev) - log_z
    w = torch.exp(log_w)
    info = float((w * (log_l - log_z)).sum())
    info = max(info, 0.0)
    return NestedResult(log_z=log_z, log_z_err=math.sqrt(info / n_live), information=info,
                        n_iter=it, n_like=n_like, samples=samples, log_w=log_w, log_l=log_l,
                        history=history)
