"""Training the learned start of the cell inversion on a solver's own states.

The network (11 -> 64 -> 64 -> 4, GELU; kt.h, learned-start section) proposes
the start y_0 e_c of the Newton inversion of Sec. 2.4 / Sec. 3.2, e_c being
the conformal closed-form root.  Training pairs are the solver's states and
their inversion by the library; the forward pass, loss, backward pass and
Adam step are the library's kernels (kt_mlp_*), so everything here is
argument marshalling and the choice of samples.
"""
from __future__ import annotations

import math

# the start uses y_0 only; the velocity outputs are a diagnostic
LOSS_WEIGHTS = (1.0, 0.05, 0.05, 0.05)


def snapshot_pairs(solver, e_floor: float, min_e_over_floor: float = 10.0):
    """Features (11, n) and targets (4, n) of the current state's cells whose
    T^{tau tau} exceeds min_e_over_floor * e_floor.  q is regulated after the
    step's recovery, so the targets come from a fresh inversion of q."""
    f = solver.fields(("q",))
    q = f["q"].reshape(15, -1)
    keep = q[0] > min_e_over_floor * e_floor
    ins = [q[k][keep].contiguous() for k in (0, 1, 2, 3, 4, 5, 6, 7, 14)]
    tau = solver.observables()["tau"]
    e, u, _, _ = solver.recover(ins, tau, with_iters=False)
    return solver.mlp_features(ins, tau, e, u)


def collect_pairs(solver, e_floor: float, n_snap: int, steps_between: int, max_pairs: int | None = None,
                  seed: int = 0):
    """Pairs from n_snap snapshots taken steps_between steps apart (the solver
    advances n_snap * steps_between steps), subsampled to max_pairs."""
    torch = solver.torch
    xs, ts = [], []
    for _ in range(n_snap):
        x, t = snapshot_pairs(solver, e_floor)
        xs.append(x)
        ts.append(t)
        solver.step(steps_between)
    X, T = torch.cat(xs, 1), torch.cat(ts, 1)
    if max_pairs is not None and X.shape[1] > max_pairs:
        gen = torch.Generator(device=X.device)
        gen.manual_seed(seed)
        idx = torch.randperm(X.shape[1], device=X.device, generator=gen)[:max_pairs]
        X, T = X[:, idx].contiguous(), T[:, idx].contiguous()
    return X, T


def train(solver, X, T, steps: int, batch: int = 8192, lr: float = 2e-3, seed: int = 0,
          record_every: int = 100):
    """Adam on minibatches drawn with replacement, step size decaying on a
    cosine from lr to lr/10.  Returns the losses at the first step and every
    record_every steps."""
    torch = solver.torch
    gen = torch.Generator(device=X.device)
    gen.manual_seed(seed)
    losses = []
    for it in range(1, steps + 1):
        idx = torch.randint(0, X.shape[1], (batch,), device=X.device, generator=gen)
        xb, tb = X[:, idx].contiguous(), T[:, idx].contiguous()
        y, act = solver.mlp_fwd(xb, keep_act=True)
        L, dy = solver.mlp_loss(y, tb, LOSS_WEIGHTS)
        g = solver.mlp_bwd(xb, act, dy)
        solver.mlp_adam(g, it, lr=lr * (0.55 + 0.45 * math.cos(math.pi * it / steps)))
        if it == 1 or it % record_every == 0:
            losses.append(L.item())
    return losses


__all__ = ["LOSS_WEIGHTS", "snapshot_pairs", "collect_pairs", "train"]
