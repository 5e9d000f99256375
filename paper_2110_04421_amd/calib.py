"""Learned calibration of (R, S_0..S_8) from a daily incidence curve, against grid search.

The paper leaves calibration from aggregate data as the direction beyond grid search
(section 1; section 6).  Here the plain simulator generates its own training data
(batched runs with parameters drawn uniformly over R in [3, 7], S_a in [0.35, 1.47]);
the BF16 matrix-core network learns the inverse map; a prediction is judged by
re-simulating the plain simulator at the predicted parameters (independent Philox
stream) and measuring the relative L2 distance to the target curve.  Grid search over
R (S at its reference profile), and over R times one susceptibility shared by all age
groups, is the fallback and the baseline.  Gradient descent through the relaxed
simulator's adjoint (``gd_fit``), from the training mean and from the network's
prediction, is the third method.

R and the S_a enter eq. 1 only as the products rho_a = R S_a (the coefficient of
age group a is R kappa S_a), so a curve can at best identify the nine products, and
mostly their mean.  The network is therefore trained on the standardised logarithms
of the products; a prediction is split back into (R, S) with R = mean_a(rho_a) /
mean(S range) clipped to the R range and S_a = rho_a / R, which re-simulates the
predicted products exactly.

    python -m paper_2110_04421_amd.calib --train 50000 --heldout 1000 --agents 100000
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import _lib as L

R_LO, R_HI, S_LO, S_HI = 3.0, 7.0, 0.35, 1.47
NTHETA = 10


def to_unit(theta):
    t = np.asarray(theta, np.float64)
    out = np.empty_like(t)
    out[:, 0] = (t[:, 0] - R_LO) / (R_HI - R_LO)
    out[:, 1:] = (t[:, 1:] - S_LO) / (S_HI - S_LO)
    return out


def from_unit(u):
    u = np.clip(np.asarray(u, np.float64), 0.0, 1.0)
    out = np.empty_like(u)
    out[:, 0] = R_LO + u[:, 0] * (R_HI - R_LO)
    out[:, 1:] = S_LO + u[:, 1:] * (S_HI - S_LO)
    return out


S_MID = 0.5 * (S_LO + S_HI)
N_RHO = 9


def products(theta):
    """rho_a = R S_a [n, 9]: what eq. 1 sees of (R, S_0..S_8)."""
    t = np.asarray(theta, np.float64)
    return t[:, :1] * t[:, 1:]


def split_products(rho):
    """(R, S) with R S_a = rho_a: R = mean(rho) / mean of the S range, within [3, 7]."""
    rho = np.asarray(rho, np.float64)
    R = np.clip(rho.mean(1) / S_MID, R_LO, R_HI)
    return np.concatenate([R[:, None], rho / R[:, None]], 1)


def sample_theta(n, seed):
    rng = np.random.default_rng(seed)
    return np.concatenate([rng.uniform(R_LO, R_HI, (n, 1)), rng.uniform(S_LO, S_HI, (n, 9))], 1)


def simulate_curves(params, base_pop, theta, seed, stream0=0, days=180, batch=256, log=None):
    """Daily incidence [n, days] of plain runs of ``base_pop`` at each parameter row,
    ``batch`` runs per launch (replicate r uses Philox stream stream0 + r)."""
    import dataclasses
    from synthpop import replicate_population
    from .sim import Simulator
    theta = np.asarray(theta, np.float64)
    n = theta.shape[0]
    out = np.zeros((n, days), np.int64)
    p = dict(params, seed=int(seed), n_steps=days, mode=L.HARD)
    reps = {}                                  # the agents are the same for every batch
    for b0 in range(0, n, batch):
        b1 = min(n, b0 + batch)
        if b1 - b0 not in reps:
            reps[b1 - b0] = replicate_population(base_pop, b1 - b0)
        pop = dataclasses.replace(reps[b1 - b0], R=theta[b0:b1, 0].astype(np.float32),
                                  susceptibility=theta[b0:b1, 1:].astype(np.float32),
                                  stream=(stream0 + np.arange(b0, b1)).astype(np.uint32))
        with Simulator(p, pop) as s:
            out[b0:b1] = s.run(days)[:, :, L.C_NEW].T
        if log:
            log(f"simulated {b1}/{n} runs")
    return out


class Features:
    """log1p of the daily incidence, standardised per day, padded to 192 inputs."""

    def fit(self, curves):
        z = np.log1p(np.asarray(curves, np.float64))
        self.mu = z.mean(0)
        self.sd = z.std(0) + 1e-3
        return self

    def __call__(self, curves):
        z = (np.log1p(np.asarray(curves, np.float64)) - self.mu) / self.sd
        x = np.zeros((z.shape[0], L.MLP_IN), np.float32)
        x[:, :z.shape[1]] = z
        return x


class Calibrator:
    """The network maps features of a curve to the standardised log products
    log(R S_a) (nine outputs of sixteen)."""

    def __init__(self, seed=0, max_batch=1024):
        from .mlp import MLP
        self.net = MLP(max_batch, seed=seed)
        self.feat = None

    def _targets(self, theta):
        y = np.zeros((theta.shape[0], L.MLP_OUT), np.float32)
        y[:, :N_RHO] = (np.log(products(theta)) - self.zmu) / self.zsd
        return y

    def _forward_all(self, x):
        out = []
        for b0 in range(0, x.shape[0], self.net.max_batch):
            out.append(self.net.forward(x[b0:b0 + self.net.max_batch].contiguous()))
        return self.net.torch.cat(out)

    def _mse(self, x, y):
        pred = self._forward_all(x)[:, :N_RHO]
        return float(((pred - y[:, :N_RHO]) ** 2).mean().cpu())

    def train(self, curves, theta, epochs=30, batch=256, lr=1e-3, seed=0, val_frac=0.1, log=None):
        """Adam on the network's own kernels; the epoch with the lowest validation MSE
        (held-back share of the training runs) is kept."""
        import torch
        n_all = theta.shape[0]
        n_val = max(1, int(val_frac * n_all))
        self.feat = Features().fit(curves[n_val:])
        z = np.log(products(theta[n_val:]))
        self.zmu, self.zsd = z.mean(0), z.std(0) + 1e-6
        x_all = torch.from_numpy(self.feat(curves)).cuda()
        y_all = torch.from_numpy(self._targets(theta)).cuda()
        xv, yv = x_all[:n_val], y_all[:n_val]
        x, y = x_all[n_val:], y_all[n_val:]
        rng = np.random.default_rng(seed)
        n = x.shape[0]
        hist, best = [], (np.inf, None)
        for ep in range(epochs):
            perm = torch.from_numpy(rng.permutation(n)).cuda()
            tot = torch.zeros(1, dtype=torch.float32, device="cuda")
            for b0 in range(0, n - batch + 1, batch):
                idx = perm[b0:b0 + batch]
                # the loss stays on the device (stream order): one read-back an epoch
                tot += self.net.train_step(x[idx].contiguous(), y[idx].contiguous(), N_RHO, lr=lr)
            val = self._mse(xv, yv)
            hist.append((float(tot.cpu()) / max(1, n // batch), val))
            if val < best[0]:
                best = (val, (self.net.master.clone(), self.net.params.clone()))
            if log:
                log(f"epoch {ep}: train {hist[-1][0]:.4f} val {val:.4f}")
        self.net.master.copy_(best[1][0])
        self.net.params.copy_(best[1][1])
        self.best_val = best[0]
        return hist

    def predict(self, curves):
        """(R, S_0..S_8) [n, 10] whose products are the network's prediction."""
        import torch
        x = torch.from_numpy(self.feat(curves)).cuda()
        zt = self._forward_all(x)[:, :N_RHO].cpu().numpy().astype(np.float64)
        return split_products(np.exp(zt * self.zsd + self.zmu))


def rel_l2(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.linalg.norm(a - b, axis=1) / np.maximum(np.linalg.norm(b, axis=1), 1.0)


def grid_thetas(n_r=41):
    S0 = np.linspace(S_LO, S_HI, 9)
    return np.concatenate([np.linspace(R_LO, R_HI, n_r)[:, None], np.tile(S0, (n_r, 1))], 1)


def grid_fit(grid_curves, grid_theta, targets):
    """Grid point whose curve is nearest (L2 of log1p) to each target."""
    g = np.log1p(grid_curves.astype(np.float64))
    t = np.log1p(np.asarray(targets, np.float64))
    d = ((t[:, None, :] - g[None, :, :]) ** 2).sum(-1)
    return grid_theta[np.argmin(d, 1)]


def grid2_thetas(n_r=21, n_s=11):
    """Two-dimensional grid: R over [3, 7] times one susceptibility shared by every age
    group over [0.35, 1.47]."""
    R, S = np.meshgrid(np.linspace(R_LO, R_HI, n_r), np.linspace(S_LO, S_HI, n_s), indexing="ij")
    return np.concatenate([R.reshape(-1, 1), np.repeat(S.reshape(-1, 1), 9, 1)], 1)


def curve_loss(c, target):
    """Per-curve loss mean_t (log1p c - log1p c*)^2 and its derivative in c."""
    c = np.maximum(np.asarray(c, np.float64), 0.0)
    dz = np.log1p(c) - np.log1p(np.asarray(target, np.float64))
    T = c.shape[1]
    return (dz ** 2).mean(1), 2.0 * dz / (1.0 + c) / T


def gd_fit(params, base_pop, targets, theta0, seed, stream0=0, iters=30, lr=0.05, days=180,
           batch=256, tau=0.1, log=None, straight_through=False):
    """Fit (R, S_0..S_8) to each hard incidence curve by gradient descent through the
    relaxed simulator's adjoint (abm_grad); with ``straight_through`` the forward runs
    are hard and the adjoint uses the relaxed sample's derivative.

    Target r is fitted on its own Philox stream (seed, stream0 + r), so the relaxed run
    shares the noise of the run that made the curve.  Adam on the unit scale, projected
    onto [0, 1], with the step decaying geometrically to a tenth of ``lr`` over the
    iterations; the loss is ``curve_loss`` of the relaxed incidence.  The relaxation
    temperature ``tau`` is kept small: the relaxed infection mass of an agent with a
    small p averages about p * pi tau / sin(pi tau) (1.57 p at tau = 0.5, 1.02 p at
    tau = 0.1), so a warm relaxation fits a different epidemic.  One soft
    simulator per batch of targets, rewound with new parameters (abm_set_theta) at
    every step.  Returns the iterate of lowest loss per target, the mean loss per step
    and the mean over targets of each one's lowest loss."""
    import dataclasses
    from synthpop import replicate_population
    from .sim import Simulator
    targets = np.asarray(targets, np.float64)
    theta0 = np.asarray(theta0, np.float64)
    n = targets.shape[0]
    scale = np.array([R_HI - R_LO] + [S_HI - S_LO] * 9)
    p = dict(params, seed=int(seed), n_steps=days, mode=L.SOFT, gumbel_tau=float(tau))
    best_th = theta0.copy()
    best_all = np.zeros(n)
    hist = np.zeros(iters)
    for b0 in range(0, n, batch):
        b1 = min(n, b0 + batch)
        pop = dataclasses.replace(replicate_population(base_pop, b1 - b0),
                                  R=theta0[b0:b1, 0].astype(np.float32),
                                  susceptibility=theta0[b0:b1, 1:].astype(np.float32),
                                  stream=(stream0 + np.arange(b0, b1)).astype(np.uint32))
        u = to_unit(theta0[b0:b1])
        m = np.zeros_like(u)
        v = np.zeros_like(u)
        best = np.full(b1 - b0, np.inf)
        with Simulator(p, pop, straight_through=straight_through) as sim:
            for it in range(iters):
                th = from_unit(u)
                sim.set_theta(th)
                c = sim.run(days)
                loss, dl = curve_loss(c, targets[b0:b1])
                better = loss < best
                best[better] = loss[better]
                best_th[b0:b1][better] = th[better]
                hist[it] += loss.sum()
                g = sim.grad(dl.astype(np.float32)).astype(np.float64) * scale
                m = 0.9 * m + 0.1 * g
                v = 0.999 * v + 0.001 * g * g
                mh, vh = m / (1 - 0.9 ** (it + 1)), v / (1 - 0.999 ** (it + 1))
                step = lr * 0.1 ** (it / max(1, iters - 1))
                u = np.clip(u - step * mh / (np.sqrt(vh) + 1e-8), 0.0, 1.0)
        best_all[b0:b1] = best
        if log:
            log(f"gradient fit {b1}/{n}: mean loss {best.mean():.4f}")
    return best_th, hist / n, float(best_all.mean())


def matched_grid2_thetas(n_runs):
    """A two-dimensional grid (R x one shared susceptibility) of about ``n_runs``
    points, twice as many R values as susceptibility values: grid search given the
    simulations the network's training set took."""
    n_s = max(2, int(round(np.sqrt(n_runs / 2.0))))
    return grid2_thetas(n_r=max(2, n_runs // n_s), n_s=n_s)


def run(n_train=50000, n_heldout=1000, n_agents=100_000, epochs=30, days=180, batch=256,
        log=None, tol=None, n_gd=256, gd_iters=30, matched_grid=True):
    """The whole calibration study; returns a summary dict.

    Held-out targets: seed 2, stream words 0..n-1.  Each prediction is re-simulated
    twice: on the target's own stream (common random numbers: isolates the parameter
    error; the true parameters give 0) and on an independent stream (seed 3; the true
    parameters give the noise floor).  Grid search runs on seed 4: the 41-point R grid,
    the 231-point R x shared-susceptibility grid and (``matched_grid``) a grid of that
    form with as many points as the network's training runs."""
    from synthpop import workload
    p, pop = workload(4, n=n_agents, mode=L.HARD, n_steps=days)
    t0 = time.perf_counter()
    th_tr = sample_theta(n_train, 11)
    c_tr = simulate_curves(p, pop, th_tr, seed=1, days=days, batch=batch, log=log)
    t_data = time.perf_counter() - t0
    th_ho = sample_theta(n_heldout, 22)
    c_ho = simulate_curves(p, pop, th_ho, seed=2, days=days, batch=batch, log=log)
    t0 = time.perf_counter()
    cal = Calibrator()
    hist = cal.train(c_tr, th_tr, epochs=epochs, log=log)
    t_train = time.perf_counter() - t0
    t0 = time.perf_counter()
    th_mlp = cal.predict(c_ho)
    t_pred = time.perf_counter() - t0
    fits = {"mlp": th_mlp}
    seconds = dict(training_data=t_data, training=t_train, mlp_predict=t_pred)
    runs = dict(mlp=n_train)
    grids = [("grid", grid_thetas()), ("grid2d", grid2_thetas())]
    if matched_grid:
        grids.append(("grid2d_matched", matched_grid2_thetas(n_train)))
    for name, gt in grids:
        t0 = time.perf_counter()
        if log:
            log(f"grid search {name}: {gt.shape[0]} runs")
        fits[name] = grid_fit(simulate_curves(p, pop, gt, seed=4, days=days, batch=batch, log=log), gt, c_ho)
        seconds[name + "_search"] = time.perf_counter() - t0
        runs[name] = int(gt.shape[0])
    th_mean = np.tile(th_tr.mean(0), (n_heldout, 1))
    fits["training_mean_params"] = th_mean
    sim = lambda th, seed: simulate_curves(p, pop, th, seed=seed, days=days, batch=batch, log=log)
    if log:
        log("re-simulating every fit on the independent and the targets' own streams")
    e_ind = {k: rel_l2(sim(th, 3), c_ho) for k, th in list(fits.items()) + [("true_params", th_ho)]}
    e_crn = {k: rel_l2(sim(th, 2), c_ho) for k, th in fits.items()}
    unit = lambda th: float(np.sqrt(((to_unit(th) - to_unit(th_ho)) ** 2).mean()))
    rmse_R = lambda th: float(np.sqrt(((th[:, 0] - th_ho[:, 0]) ** 2).mean()))
    lrho = lambda th: np.log(products(th))
    rho_rmse = lambda th: float(np.sqrt(((lrho(th) - lrho(th_ho)) ** 2).mean()))
    rbar = lambda th: np.log(products(th).mean(1))
    rbar_rmse = lambda th: float(np.sqrt(((rbar(th) - rbar(th_ho)) ** 2).mean()))
    summary = dict(
        agents=n_agents, days=days, train_runs=n_train, heldout=n_heldout, epochs=epochs,
        simulations_per_method=runs,
        train_mse_first=hist[0][0], train_mse_last=hist[-1][0], best_val_mse=cal.best_val,
        resim_rel_l2_independent_stream={k: float(v.mean()) for k, v in e_ind.items()},
        resim_rel_l2_same_stream={k: float(v.mean()) for k, v in e_crn.items()},
        resim_rel_l2_same_stream_median={k: float(np.median(v)) for k, v in e_crn.items()},
        transmissibility_rmse_log={k: rbar_rmse(th) for k, th in fits.items()},
        products_rmse_log={k: rho_rmse(th) for k, th in fits.items()},
        param_rmse_unit={k: unit(th) for k, th in fits.items()},
        R_rmse={k: rmse_R(th) for k, th in fits.items()},
        seconds=seconds)
    if n_gd > 0:
        # gradient descent through the adjoint on the first n_gd held-out curves, from
        # the training mean and from the network's prediction
        k = min(n_gd, n_heldout)
        gd = {}
        for name, th0 in (("gd_from_mean", th_mean[:k]), ("gd_from_mlp", th_mlp[:k]),
                          ("gd_from_grid2d", fits["grid2d"][:k])):
            t0 = time.perf_counter()
            th, h, lbest = gd_fit(p, pop, c_ho[:k], th0, seed=2, iters=gd_iters, days=days, batch=batch,
                                  log=log)
            gd[name] = dict(seconds=time.perf_counter() - t0, loss_first=float(h[0]), loss_best=lbest,
                            theta=th)
        sub = {n_: th[:k] for n_, th in fits.items()}
        sub.update({n_: v["theta"] for n_, v in gd.items()})
        e_sub = {n_: rel_l2(simulate_curves(p, pop, th, seed=2, days=days, batch=batch, log=log), c_ho[:k])
                 for n_, th in sub.items()}
        summary["gradient_descent"] = dict(
            targets=k, iterations=gd_iters,
            resim_rel_l2_same_stream={n_: float(v.mean()) for n_, v in e_sub.items()},
            resim_rel_l2_same_stream_median={n_: float(np.median(v)) for n_, v in e_sub.items()},
            param_rmse_unit={n_: float(np.sqrt(((to_unit(th) - to_unit(th_ho[:k])) ** 2).mean()))
                             for n_, th in sub.items()},
            relaxed_loss_start_and_best={n_: (v["loss_first"], v["loss_best"]) for n_, v in gd.items()},
            seconds={n_: v["seconds"] for n_, v in gd.items()})
    if tol is not None:
        # fallback: where the network's re-simulation misses the target by more than tol,
        # grid search runs as well and the better of the two fits is kept
        fb = e_crn["mlp"] > tol
        e_comb = np.where(fb, np.minimum(e_crn["grid2d"], e_crn["mlp"]), e_crn["mlp"])
        summary["with_fallback"] = dict(tol=tol, fallback_share=float(fb.mean()),
                                        resim_rel_l2_same_stream=float(e_comb.mean()))
    return summary


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--train", type=int, default=50000)
    ap.add_argument("--heldout", type=int, default=1000)
    ap.add_argument("--agents", type=int, default=100_000)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--days", type=int, default=180)
    ap.add_argument("--tol", type=float, default=0.5)
    ap.add_argument("--gd-targets", type=int, default=256)
    ap.add_argument("--gd-iters", type=int, default=30)
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)
    log = lambda m: print(f"[calib {time.strftime('%H:%M:%S')}] {m}", file=sys.stderr, flush=True)
    s = run(a.train, a.heldout, a.agents, a.epochs, a.days, log=log, tol=a.tol, n_gd=a.gd_targets,
            gd_iters=a.gd_iters)
    txt = json.dumps(s, indent=1)
    print(txt)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")


if __name__ == "__main__":
    main()
