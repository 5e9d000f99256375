"""Relaxed (differentiable) version of the daily step, in FP64, with forward-mode
tangents for the gradient with respect to (R, S_0..S_8) of every replicate.

The paper leaves gradient-based calibration of the simulator's parameters as its
motivation and future direction (abstract; section 1; section 6), without an
algorithm.  The relaxation used here keeps eqs. 1-2 and the contact graph, and
replaces the hard infection draw u < p by a Gumbel-softmax (binary concrete) sample
with the same uniform u:

    y_j = sigmoid((logit p_j - logit u_j) / tau_g),  logit p = log(expm1(lambda dt)),

so that y -> [u < p] as tau_g -> 0.  Each agent carries a susceptible mass s_j;
the mass exposed on day t is e_j(t) = s_j(t) y_j(t), s_j(t+1) = s_j(t) - e_j(t).
Infectiousness on day t: inf_i(t) = sum_tau Atab[tau] e_i(t - tau) (initial
infections: e = 1 on day -1).  lambda_j(t) = R kappa S[a_j] sum_{e in row j} w_e
inf_src(t).  Daily relaxed incidence c_r(t) = sum_{j in r} e_j(t).
Interventions are off in this mode.

Tangents are propagated alongside every quantity (dual numbers with 10 components,
one per parameter of the agent's own replicate).

Straight-through variant (``straight_through``): the forward pass takes the hard
sample [u < p] (the relaxed sample's sign, z > 0), so the state follows the hard step,
and the tangent of the sample is still the relaxed one's, y(1 - y)/tau_g dz.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import philox
from .graph import build_graph, static_maps
from .step import f32, f32v
from .tables import infectiousness_table

NTHETA = 10


def sigmoid(z):
    return np.where(z >= 0, 1.0 / (1.0 + np.exp(-np.abs(z))), np.exp(-np.abs(z)) / (1.0 + np.exp(-np.abs(z))))


class SoftModel:
    def __init__(self, pop, params, R=None, S=None, straight_through=False):
        self.pop = pop
        self.st = bool(straight_through)
        self.p = dict(params)
        self.maps = static_maps(pop)
        self.N = int(pop.agent_offset[-1])
        self.nrep = int(pop.agent_offset.size - 1)
        self.rep = self.maps["rep"]
        self.loc = self.maps["local"]
        self.word = self.maps["stream"]
        self.age = np.asarray(pop.age, np.int64)
        p = self.p
        self.Atab = np.array(infectiousness_table(float(p["gamma_shape"]), float(p["gamma_scale"]),
                                                  int(p["e_days"]), int(p["i_days"]),
                                                  [float(a) for a in p["A_stage"]]))
        self.L = int(p["e_days"]) + int(p["i_days"])
        self.R = f32v(pop.R) if R is None else np.asarray(R, np.float64)
        self.S = f32v(pop.susceptibility) if S is None else np.asarray(S, np.float64)
        self.kappa = f32(p["kappa"])
        self.tau = f32(p["gumbel_tau"])
        self.dt = f32(p["dt"])

    def coef(self):
        """coef_j = R kappa S[a_j] and its tangent [N, 10] (d/dR, d/dS_0..S_8)."""
        Rj = self.R[self.rep]
        Sj = self.S[self.rep, self.age]
        c = Rj * self.kappa * Sj
        cd = np.zeros((self.N, NTHETA))
        cd[:, 0] = self.kappa * Sj
        cd[np.arange(self.N), 1 + self.age] = Rj * self.kappa
        return c, cd

    def logit_u(self, t):
        w = philox.draw_words(int(self.p["seed"]), self.loc, t, self.word, philox.PURPOSE_AGENT, 0)[0]
        u = philox.uniform(w)
        return np.log(u) - np.log1p(-u)

    def run(self, T, tangents=True, record=False):
        """Relaxed run of T days: c [R, T], c_dot [R, T, 10] (zeros if not tangents)."""
        N = self.N
        coef, coef_d = self.coef()
        s = np.ones(N)
        s_d = np.zeros((N, NTHETA))
        hist = {}                              # day -> (e [N], e_dot [N, 10])
        seeds = np.asarray(self.pop.initial_infected, np.int64)
        e0 = np.zeros(N)
        e0[seeds] = 1.0
        s[seeds] = 0.0
        hist[-1] = (e0, np.zeros((N, NTHETA)))
        c = np.zeros((self.nrep, T))
        c_d = np.zeros((self.nrep, T, NTHETA))
        rec = []
        for t in range(T):
            inf = np.zeros(N)
            inf_d = np.zeros((N, NTHETA))
            for tau in range(1, self.L + 1):
                if t - tau in hist:
                    e, ed = hist[t - tau]
                    inf += self.Atab[tau] * e
                    if tangents:
                        inf_d += self.Atab[tau] * ed
            rp, col, w, _ = build_graph(self.pop, self.p, t, self.maps)
            A = sp.csr_matrix((w, col, rp), shape=(N, N))
            sigma = A @ inf
            lam = coef * sigma
            x = lam * self.dt
            pos = x > 0
            y = np.zeros(N)
            ell = np.log(np.expm1(x[pos]))
            lu = self.logit_u(t)
            y[pos] = sigmoid((ell - lu[pos]) / self.tau)
            yf = y                             # the sample the state takes
            if self.st:
                yf = np.zeros(N)
                yf[pos] = (ell - lu[pos] > 0).astype(np.float64)
            e = s * yf
            if tangents:
                sigma_d = A @ inf_d
                lam_d = coef_d * sigma[:, None] + coef[:, None] * sigma_d
                dy = np.zeros(N)
                p = -np.expm1(-x[pos])
                dy[pos] = y[pos] * (1 - y[pos]) / self.tau / p * self.dt
                y_d = dy[:, None] * lam_d
                e_d = s_d * yf[:, None] + s[:, None] * y_d
            else:
                e_d = np.zeros((N, NTHETA))
            if record:
                rec.append(dict(sigma=sigma, lam=lam, y=y, s=s.copy(), e=e))
            c[:, t] = np.bincount(self.rep, weights=e, minlength=self.nrep)
            if tangents:
                for k in range(NTHETA):
                    c_d[:, t, k] = np.bincount(self.rep, weights=e_d[:, k], minlength=self.nrep)
            s = s - e
            s_d = s_d - e_d
            hist[t] = (e, e_d)
            hist.pop(t - self.L - 1, None)
        return c, c_d, rec


def gradient(c_d, dL):
    """dL/dtheta [R, 10] from the incidence tangents and dL/dc [R, T]."""
    return np.einsum("rt,rtk->rk", np.asarray(dL, np.float64), c_d)
