"""Growth-rate surrogate: a network trained on runs of the solver itself, with the solver kept as
the fallback and the reference for its error.

Inputs (supersaturation U0, seed radius R, inflow velocity u_in, time t) -> 16 crystal extents
L_k(t) along the directions 2 pi k / 16 and the 16 growth rates G_k(t) (least-squares slope of L_k
against time over the samples in [t/2, t], Section 4.1.2's linear fit on a growing window), as a
mean and a log-variance head each. Training data: batched solver runs (lbcg_batch_*) of 2-D
forced-convection instances whose (U0, R, u_in) are drawn as in the parametric sweep; training
and inference run in the library's bf16-MFMA MLP kernels (lbcg_mlp_*). A prediction whose
predicted relative growth-rate error (two standard deviations of the predicted G_k over the mean
predicted G) exceeds the calibrated threshold falls back to the solver.

The domain side is not among the four inputs, so the runs share one side length
(workloads.SURROGATE_SIDE): on domains of mixed sizes small domains deplete the supersaturation
within the run and the same four inputs give different rates. A model that also takes the side
(`with_side=True`) can be trained on the sweep's mixed sides for comparison.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import workloads as W

K_DIRS = 16
WIDTHS = [4, 256, 256, 256, 4 * K_DIRS]  # 32 means + 32 log-variances


def features(U0, R, u_in, t, t_end, side=None):
    """Affine map of the inputs onto about [-1, 1] (the domain side only for the diagnostic model
    that is given it)."""
    cols = [(np.asarray(U0) - 0.225) / 0.175, (np.asarray(R) - 10.0) / 6.0,
            (np.asarray(u_in) - 0.015) / 0.015, 2.0 * np.asarray(t) / t_end - 1.0]
    if side is not None:
        cols.append((np.asarray(side) - 160.0) / 96.0)
    return np.stack(cols, axis=-1)


def windowed_slopes(t, L):
    """G[j, k] = least-squares slope of L[a .. j, k] against t over the samples with t >= t_j / 2
    (at least two samples)."""
    S = L.shape[0]
    G = np.zeros_like(L)
    for j in range(1, S):
        a = min(int(np.searchsorted(t, 0.5 * t[j])), j - 1)
        tt = t[a:j + 1]
        LL = L[a:j + 1]
        tm = tt.mean()
        G[j] = ((tt - tm)[:, None] * (LL - LL.mean(axis=0))).sum(axis=0) / ((tt - tm) ** 2).sum()
    G[0] = G[1]
    return G


@dataclass
class Dataset:
    draws: np.ndarray   # [n, 4]: side, U0, R, u_in
    t: np.ndarray       # [S]
    L: np.ndarray       # [n, S, K]
    G: np.ndarray       # [n, S, K]
    solve_s: float      # wall time of the solver runs


def generate(draws, steps: int = 4000, every: int = 100, group: int = 256) -> Dataset:
    """Run the solver on every draw (batched, `group` instances per launch) and record L_k(t)."""
    import torch

    from . import lbcg
    dirs = W.directions(K_DIRS)
    S = steps // every + 1
    n = len(draws)
    L = np.zeros((n, S, K_DIRS))
    t0 = time.perf_counter()
    for g0 in range(0, n, group):
        sub = draws[g0:g0 + group]
        b = lbcg.Batch([W.sweep_instance(*d) for d in sub], "fp32")
        L[g0:g0 + len(sub), 0] = b.measure(dirs)
        hist = b.run(steps, every, dirs)
        L[g0:g0 + len(sub), 1:] = np.transpose(hist, (1, 0, 2))
        b.close()
        del b
    torch.cuda.synchronize()
    solve_s = time.perf_counter() - t0
    t = np.arange(S, dtype=np.float64) * every
    G = np.stack([windowed_slopes(t, L[i]) for i in range(n)])
    return Dataset(np.asarray(draws, dtype=np.float64), t, L, G, solve_s)


def rows(ds: Dataset, with_side: bool = False):
    """Flatten (run, time) pairs into network rows: X [n S, 4 (or 5)], Y [n S, 2K]."""
    n, S, _ = ds.L.shape
    d = ds.draws
    X = features(np.repeat(d[:, 1], S), np.repeat(d[:, 2], S), np.repeat(d[:, 3], S), np.tile(ds.t, n), ds.t[-1],
                 np.repeat(d[:, 0], S) if with_side else None)
    Y = np.concatenate([ds.L.reshape(n * S, -1), ds.G.reshape(n * S, -1)], axis=1)
    return X, Y


class Surrogate:
    def __init__(self, seed: int = 0, max_batch: int = 4096, with_side: bool = False):
        from . import lbcg
        self.with_side = with_side
        self.widths = [5 if with_side else 4] + WIDTHS[1:]
        self.net = lbcg.MLP(self.widths, max_batch)
        rng = np.random.default_rng(seed)  # weight init: N(0, 1/fan_in), biases 0
        flat = []
        for i, o in zip(self.widths[:-1], self.widths[1:]):
            flat.append((rng.normal(size=(o, i)) / math.sqrt(i)).ravel())
            flat.append(np.zeros(o))
        self.net.set_params(np.concatenate(flat).astype(np.float32))
        self.max_batch = max_batch
        self.mean = None
        self.std = None
        self.t_end = None

    def train(self, ds: Dataset, steps: int = 3000, batch: int = 1024, lr: float = 2e-3, seed: int = 1,
              log=None):
        import torch
        X, Y = rows(ds, self.with_side)
        self.t_end = float(ds.t[-1])
        self.mean = Y.mean(axis=0)
        self.std = Y.std(axis=0) + 1e-9
        Xd = torch.tensor(X, dtype=torch.float32, device="cuda")
        Td = torch.tensor((Y - self.mean) / self.std, dtype=torch.float32, device="cuda")
        rng = np.random.default_rng(seed)
        nrow = X.shape[0]
        # every step's rows (a fresh permutation per epoch, the tail that does not fill a batch
        # skipped), uploaded once so that the steps queue up without host round trips
        batches = np.empty((steps, min(batch, nrow)), dtype=np.int32)
        perm = rng.permutation(nrow)
        pos = 0
        for k in range(steps):
            if pos + batch > nrow:
                perm = rng.permutation(nrow)
                pos = 0
            batches[k] = perm[pos:pos + batch]
            pos += batch
        idx_all = torch.tensor(batches, device="cuda")
        losses = []
        t0 = time.perf_counter()
        for k in range(steps):
            lr_k = lr * (0.1 if k >= 0.75 * steps else 1.0)
            want = k >= steps - 50 or (log is not None and k % 500 == 0)  # the loss costs a synchronisation
            loss = self.net.train_step(Xd, Td, idx_all[k], lr=lr_k, want_loss=want)
            if want:
                losses.append(loss)
            if log and (k % 500 == 0 or k == steps - 1):
                log(f"surrogate step {k}: loss {losses[-1]:.4f}")
        torch.cuda.synchronize()
        return dict(train_s=time.perf_counter() - t0, final_loss=float(np.mean(losses[-50:])), steps=steps,
                    rows=nrow, batch=batch)

    def predict(self, draws, t):
        """Means and standard deviations of L_k and G_k in physical units: 4 arrays [n, len(t), K]."""
        import torch
        d = np.asarray(draws, dtype=np.float64)
        n, S = d.shape[0], len(t)
        X = features(np.repeat(d[:, 1], S), np.repeat(d[:, 2], S), np.repeat(d[:, 3], S), np.tile(t, n), self.t_end,
                     np.repeat(d[:, 0], S) if self.with_side else None)
        out = []
        for a in range(0, X.shape[0], self.max_batch):
            xd = torch.tensor(X[a:a + self.max_batch], dtype=torch.float32, device="cuda")
            out.append(self.net.forward(xd).cpu().numpy())
        Y = np.concatenate(out).astype(np.float64)
        D = 2 * K_DIRS
        mu = Y[:, :D] * self.std + self.mean
        sd = np.exp(0.5 * np.clip(Y[:, D:], -12, 12)) * self.std
        mu = mu.reshape(n, S, D)
        sd = sd.reshape(n, S, D)
        return mu[..., :K_DIRS], sd[..., :K_DIRS], mu[..., K_DIRS:], sd[..., K_DIRS:]


def growth_error(G_pred, G_true, floor):
    """max_k |G_pred - G_true| / max(mean_k G_true, floor), per run (last axis = directions)."""
    return np.abs(G_pred - G_true).max(axis=-1) / np.maximum(G_true.mean(axis=-1), floor)


def subset(ds: Dataset, idx) -> Dataset:
    idx = np.asarray(idx)
    return Dataset(ds.draws[idx], ds.t, ds.L[idx], ds.G[idx], ds.solve_s * len(idx) / len(ds.draws))


def final_errors(model: Surrogate, ds: Dataset, floor: float, criterion: str = "max_dir"):
    """(predicted, true) relative growth-rate errors of the runs in ds at their final time.

    criterion "max_dir": error = max_k |G_pred,k - G_k| / mean_k G_k (every direction);
    criterion "avg": error = |mean_k G_pred,k - mean_k G_k| / mean_k G_k (the average growth rate
    G_th of the paper's tables). The predicted error is two predicted standard deviations over
    the predicted mean growth rate (for "avg", the mean of the per-direction deviations)."""
    _, _, Gm, Gs = model.predict(ds.draws, ds.t[-1:])
    Gm, Gs = Gm[:, 0], Gs[:, 0]
    Gt = ds.G[:, -1]
    den_pred = np.maximum(np.abs(Gm.mean(axis=-1)), floor)
    den_true = np.maximum(Gt.mean(axis=-1), floor)
    if criterion == "avg":
        return 2.0 * Gs.mean(axis=-1) / den_pred, np.abs(Gm.mean(axis=-1) - Gt.mean(axis=-1)) / den_true
    return 2.0 * Gs.max(axis=-1) / den_pred, np.abs(Gm - Gt).max(axis=-1) / den_true


def threshold_from(pred, true, tol: float) -> float:
    """The largest predicted-error threshold (at most tol) under which every run it accepts has a
    true error within tol: the runs sorted by predicted error are accepted up to the first miss
    (0 if the most confident run already misses)."""
    pred, true = np.asarray(pred, dtype=float), np.asarray(true, dtype=float)
    order = np.argsort(pred, kind="stable")
    ok = np.cumprod(true[order] <= tol).astype(bool)
    if not ok.any():
        return 0.0
    last = int(np.nonzero(ok)[0].max())
    thr = float(pred[order][last])
    if last + 1 < len(order) and pred[order][last + 1] == thr:  # a tie with the first miss
        thr = float(np.nextafter(thr, -np.inf))
    return min(thr, tol)


def calibrate(model: Surrogate, cal: Dataset, tol: float, floor: float, criterion: str = "max_dir") -> float:
    """Acceptance threshold from calibration runs the model was not trained on (threshold_from)."""
    pred, true = final_errors(model, cal, floor, criterion)
    return threshold_from(pred, true, tol)


def evaluate(model: Surrogate, held: Dataset, tol: float = 0.05, floor: float = None, criterion: str = "max_dir",
             threshold: float = None):
    """Predict the final growth rates of held-out draws, accept those whose predicted error is at
    most `threshold` (default: tol), and fall back to the solver for the rest (timed with the
    batched solver). Errors as in final_errors.

    The solver alone is timed on all held-out draws just before the fallback, so that both run in
    the same state of the device and its allocator."""
    import torch
    if floor is None:
        floor = 0.1 * float(np.abs(held.G[:, -1]).mean())
    thr = tol if threshold is None else threshold
    all_draws = [tuple(d) for d in held.draws]
    steps, every = int(held.t[-1]), int(held.t[1] - held.t[0])
    t_alone = generate(all_draws, steps=steps, every=every).solve_s
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pred_err, true_err = final_errors(model, held, floor, criterion)
    torch.cuda.synchronize()
    t_infer = time.perf_counter() - t0
    accept = pred_err <= thr
    n = len(held.draws)
    n_fb = int((~accept).sum())
    t_fb = 0.0
    if n_fb:  # the rejected draws through the batched solver: their results are the solver's
        t_fb = generate([tuple(d) for d in held.draws[~accept]], steps=steps, every=every).solve_s
    err_final = np.where(accept, true_err, 0.0)
    total = t_infer + t_fb
    q = lambda v: None if v is None else round(float(v), 5)
    return dict(criterion=criterion, held_out=n, accepted=int(accept.sum()), fallback=n_fb, floor=floor, tol=tol,
                threshold=q(thr), infer_s=t_infer, fallback_s=t_fb, runs_per_s=n / total if total > 0 else float("inf"),
                accepted_err_max=q(true_err[accept].max()) if accept.any() else None,
                accepted_err_mean=q(true_err[accept].mean()) if accept.any() else None,
                accepted_within_tol=q((true_err[accept] <= tol).mean()) if accept.any() else None,
                all_err_median=q(np.median(true_err)), all_err_p90=q(np.quantile(true_err, 0.9)),
                delivered_err_max=q(err_final.max()), solver_alone_runs_per_s=n / t_alone)


def run_study(n_train: int = 4096, n_held: int = 256, steps: int = 4000, train_steps: int = 12000, log=None,
              seed_train: int = 22060, seed_held: int = 22061, mixed_sides: bool = False):
    """Generate the training and held-out runs (one domain side, workloads.surrogate_draws), train
    the four-input model, evaluate it with fallback. mixed_sides: also the comparison on the
    sweep's mixed domain sides, with and without the side as a fifth input."""
    cases = [("deployed", W.surrogate_draws, False, "max_dir")]
    if mixed_sides:
        cases += [("mixed_sides_with_side", W.sweep_draws, True, "max_dir"),
                  ("mixed_sides_four_inputs", W.sweep_draws, False, "max_dir")]
    out = dict(train_runs=n_train, held_out_runs=n_held, steps=steps, side=W.SURROGATE_SIDE)
    data = {}
    for name, drawfn, ws, crit in cases:
        if drawfn not in data:
            tr = generate(drawfn(n_train, seed=seed_train), steps=steps)
            ho = generate(drawfn(n_held, seed=seed_held), steps=steps)
            if log:
                log(f"surrogate data ({drawfn.__name__}): {n_train} training runs solved in {tr.solve_s:.1f} s")
            data[drawfn] = (tr, ho)
        tr, ho = data[drawfn]
        # the last tenth of the training runs calibrates the acceptance threshold and is not trained on
        n_cal = max(1, n_train // 10)
        fit, cal = subset(tr, np.arange(n_train - n_cal)), subset(tr, np.arange(n_train - n_cal, n_train))
        floor = 0.1 * float(np.abs(cal.G[:, -1]).mean())
        m = Surrogate(with_side=ws)
        info = m.train(fit, steps=train_steps)
        thr = calibrate(m, cal, 0.05, floor, crit)
        res = evaluate(m, ho, floor=floor, criterion=crit, threshold=thr)
        res.update(train_s=info["train_s"], final_loss=info["final_loss"], inputs=5 if ws else 4,
                   train_runs=n_train - n_cal, calibration_runs=n_cal, solve_train_s=tr.solve_s,
                   domain="one side" if drawfn is W.surrogate_draws else "mixed sides")
        out[name] = res
        if log:
            log(f"surrogate {name}: threshold {res['threshold']}, accepted {res['accepted']}/{n_held}, "
                f"accepted err max {res['accepted_err_max']}, median err {res['all_err_median']}, "
                f"{res['runs_per_s']:.0f} runs/s vs solver {res['solver_alone_runs_per_s']:.0f}")
        m.net.close()
    return out
