"""BOAC outer loop (the method's steps 1-6) over the batched GPU evaluator.

  1. an initial design of candidates drawn uniformly in the search box;
  2-3. every candidate is rasterised, reconstructed with a fixed number of MLEM iterations and scored
     by the negative log-likelihood J, a batch at a time on the GPU (boac_objective, or
     boac_objective_grad_ex when a gradient is wanted);
  4. the observations (unit-box coordinates, J) are fitted by the GP surrogate of Eqs. (7)-(8)
     (boac_gp_fit, native FP64 on the host);
  5. new candidates maximise the expected improvement of Eqs. (9)-(10), found by a chaotic search driven
     by the logistic map z <- 4 z (1 - z): a global stage over the whole box, then local stages around
     several incumbents with geometrically shrinking radii. A batch of proposals is taken greedily from
     every evaluated point in decreasing EI, each at least `exclusion` (unit-box distance) from those
     already taken. The search runs on the GPU (boac_gp_chaos_search; chaotic_acquire is the same
     search on the host around boac_gp_ei);
  6. the largest EI is recorded each cycle; the loop stops when it falls below `ei_stop` (relative to
     the surrogate's scale) or after the given number of cycles.

Gradient-aware variant (gradient="envelope" or "unrolled"): candidates are evaluated with dJ/dtheta,
and each cycle part of the batch is a line search along -grad J from the best observations (several
step lengths, evaluated in the same batched call). The plain loop (gradient=None) is the baseline.

Every cycle is appended to a JSON-lines journal; a loop created on an existing journal replays it and
continues with the proposals an uninterrupted run would have made (the random streams are derived from
(seed, cycle)). The host does only orchestration: model fitting is native, acquisition and candidate
evaluation run in the library's kernels.
"""
from __future__ import annotations

import json
import os
import time
from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import torch

from .api import Context, Geometry, gp_fit

# search box of the head parameters (c_0..c_5 cm, mu_b, mu_c 1/cm)
DEFAULT_LO = np.array([6.5, -1.5, -1.5, -1.5, -1.5, -1.5, 0.13, 0.20])
DEFAULT_HI = np.array([8.5, 1.5, 1.5, 1.5, 1.5, 1.5, 0.17, 0.30])
LENGTH_GRID = np.geomspace(0.03, 3.0, 16)
LINE_STEPS = (0.005, 0.01, 0.02, 0.04, 0.08, 0.16)


def greedy_select(U: np.ndarray, score: np.ndarray, q: int, exclusion: float, taken=None,
                  chunk: int = 8192) -> List[int]:
    """Indices of up to q rows of U in decreasing score, each at least `exclusion` from every row taken
    before (and from the rows of `taken`). Ties keep the lower index first. Candidates are screened a
    chunk at a time against `taken` and the earlier picks (one distance matrix per chunk)."""
    order = np.argsort(-np.asarray(score, np.float64), kind="stable")
    d = U.shape[1]
    ex2 = exclusion * exclusion
    prev = np.asarray(taken, np.float64).reshape(-1, d) if taken is not None else np.empty((0, d))
    chosen: List[int] = []
    picked = np.empty((0, d))
    for c0 in range(0, len(order), chunk):
        if len(chosen) >= q:
            break
        idx = order[c0:c0 + chunk]
        idx = idx[np.isfinite(score[idx])]
        if not len(idx):
            break
        P = U[idx]
        ref = np.vstack([prev, picked])
        if len(ref):
            # |p - r|^2 = |p|^2 + |r|^2 - 2 p.r for the whole chunk at once
            d2 = (np.sum(P * P, axis=1)[:, None] + np.sum(ref * ref, axis=1)[None, :] - 2.0 * (P @ ref.T)).min(axis=1)
            keep = d2 >= ex2
            idx, P = idx[keep], P[keep]
        # accept the best remaining point of the chunk, drop its neighbours, repeat
        while len(idx) and len(chosen) < q:
            u = P[0]
            chosen.append(int(idx[0]))
            picked = np.vstack([picked, u[None, :]])
            keep = np.sum((P[1:] - u) ** 2, axis=1) >= ex2
            idx, P = idx[1:][keep], P[1:][keep]
        if not np.all(np.isfinite(score[order[c0:c0 + chunk]])):
            break
    return chosen


def _select_top(U, score, q, exclusion, taken, pool_per_pick: int = 16):
    """greedy_select over the k best scores (ties by lower index), k = pool_per_pick * q growing 4-fold
    until q picks qualify: the same picks as over everything, which is the last resort."""
    order = np.argsort(-np.asarray(score, np.float64), kind="stable")
    k = pool_per_pick * q
    while len(score) > k:
        top = np.sort(order[:k])
        pick = greedy_select(U[top], score[top], q, exclusion, taken)
        if len(pick) == q:
            return [int(top[i]) for i in pick]
        k *= 4
    return greedy_select(U, score, q, exclusion, taken)


def chaotic_acquire(ei_of, z: np.ndarray, q: int, taken, *, n_global: int, n_local: int, centres: int,
                    radius0: float, shrink: float, exclusion: float, per_step: int, local=None):
    """Step 5's search for q proposals maximising the acquisition ei_of (rows of a [m, d] unit-box array
    -> [m] values), from the chains z [P, d] in (0, 1) of the logistic map z <- 4 z (1 - z).

    Global stage: n_global rounds over the chains' points. Centres: the best evaluated points at least
    `exclusion` apart, max(centres, q) of them. Local stage: n_local rounds; chains split evenly over the
    centres sample boxes of half-width radius0 shrink^t around them, and a centre moves to its best point
    of a round when that beats it. Each round keeps its per_step best points (ties by lower index); the
    proposals are taken greedily from that pool, each at least `exclusion` from the points taken and from
    `taken`. Returns (proposals [<= q, d], largest value evaluated, number of evaluations).

    The global stage's points do not depend on the acquisition values, so its rounds go to ei_of in one
    call (each query's value does not depend on the others). local(z, C, Ce, radius0) may run the whole
    local stage elsewhere (the device: Context.gp_chaos_local) and return its rounds' points
    [n_local, per * len(C), d] and values [n_local, per * len(C)], as the loop below would produce them."""
    z = np.array(z, dtype=np.float64)
    P, d = z.shape
    pts, vals = [], []
    n_queries = 0

    def keep(U, e):
        if len(e) > per_step:
            # the per_step best, ties by lower index: every value above the per_step-th largest, then the
            # lowest indices holding that value (a partition instead of a full sort)
            thr = np.partition(e, len(e) - per_step)[len(e) - per_step]
            above = np.flatnonzero(e > thr)
            at = np.flatnonzero(e == thr)[:per_step - len(above)]
            top = np.sort(np.concatenate([above, at]))
            U, e = U[top], e[top]
        pts.append(U.copy())
        vals.append(e)

    Zs = []
    for _ in range(n_global):
        Zs.append(z)
        z = 4.0 * z * (1.0 - z)
    if Zs:
        e_all = np.asarray(ei_of(np.concatenate(Zs)), np.float64)
        for t, Z in enumerate(Zs):
            keep(Z, e_all[t * P:(t + 1) * P])
        n_queries += P * len(Zs)
    allU, allE = np.concatenate(pts), np.concatenate(vals)
    cidx = _select_top(allU, allE, min(max(centres, q), P), exclusion, None)
    C = allU[cidx].copy()
    Ce = allE[cidx].copy()
    per = max(1, P // max(1, len(C)))
    r = radius0
    if local is not None and n_local > 0:
        U_all, e_all = local(z, C, Ce, r)
        for t in range(n_local):
            keep(np.asarray(U_all[t], np.float64), np.asarray(e_all[t], np.float64))
        n_queries += int(np.asarray(e_all).size)
        n_local = 0
    for _ in range(n_local):
        zz = z[:per * len(C)].reshape(len(C), per, d)
        U = np.clip(C[:, None, :] + r * (2.0 * zz - 1.0), 0.0, 1.0).reshape(-1, d)
        e = np.asarray(ei_of(U), np.float64)
        n_queries += len(U)
        keep(U, e)
        e2 = e.reshape(len(C), per)
        j = np.argmax(e2, axis=1)
        better = e2[np.arange(len(C)), j] > Ce
        C[better] = U.reshape(len(C), per, d)[better, j[better]]
        Ce[better] = e2[better, j[better]]
        z = 4.0 * z * (1.0 - z)
        r *= shrink
    allU, allE = np.concatenate(pts), np.concatenate(vals)
    pick = _select_top(allU, allE, q, exclusion, taken)
    return allU[pick], float(allE.max()), n_queries


def line_search_points(u0: np.ndarray, grad_u: np.ndarray, steps=LINE_STEPS) -> np.ndarray:
    """Points u0 - t grad/|grad| for each step length t, clipped to the unit box ([len(steps), d])."""
    g = np.asarray(grad_u, np.float64)
    nrm = np.linalg.norm(g)
    if not np.isfinite(nrm) or nrm == 0.0:
        return np.empty((0, u0.size))
    d = -g / nrm
    return np.clip(u0[None, :] + np.asarray(steps)[:, None] * d[None, :], 0.0, 1.0)


@dataclass
class Cycle:
    index: int
    theta: np.ndarray            # [q, 8] evaluated this cycle
    J: np.ndarray                # [q]
    grad: Optional[np.ndarray]   # [q, 8] or None
    status: np.ndarray           # [q]
    kind: List[str]              # "init" | "ei" | "line" per candidate
    max_ei: float
    length: float
    timings: dict = field(default_factory=dict)

    def to_json(self):
        return {"cycle": self.index, "theta": self.theta.tolist(), "J": self.J.tolist(),
                "grad": None if self.grad is None else self.grad.tolist(), "status": self.status.tolist(),
                "kind": self.kind, "max_ei": self.max_ei, "length": self.length, "timings": self.timings}

    @staticmethod
    def from_json(r):
        return Cycle(r["cycle"], np.asarray(r["theta"]), np.asarray(r["J"]),
                     None if r["grad"] is None else np.asarray(r["grad"]), np.asarray(r["status"]),
                     list(r["kind"]), float(r["max_ei"]), float(r["length"]), r.get("timings", {}))


class BOAC:
    def __init__(self, ctx: Context, geom: Geometry, meas: torch.Tensor, *, lo=DEFAULT_LO, hi=DEFAULT_HI,
                 delta_r: float = 0.8, n_iter: int = 30, n_init: int = 64, batch: int = 64, xi: float = 0.0,
                 seed: int = 0, chains: int = 4096, n_global: int = 16, n_local: int = 32, centres: int = 8,
                 radius0: float = 0.1, shrink: float = 0.85, exclusion: float = 0.02, ei_stop: Optional[float] = None,
                 gradient: Optional[str] = None, line_starts: int = 4, ckpt_every: int = 5, n_select: int = 256,
                 noise: float = 1e-6, journal: Optional[str] = None, device_search: bool = True):
        if gradient not in (None, "envelope", "unrolled"):
            raise ValueError("gradient must be None, 'envelope' or 'unrolled'")
        self.ctx, self.geom, self.meas = ctx, geom, meas
        self.lo, self.hi = np.asarray(lo, np.float64), np.asarray(hi, np.float64)
        self.delta_r, self.n_iter, self.n_init, self.batch = float(delta_r), int(n_iter), int(n_init), int(batch)
        self.xi, self.seed = float(xi), int(seed)
        self.chains, self.n_global, self.n_local, self.centres = int(chains), int(n_global), int(n_local), int(centres)
        self.radius0, self.shrink, self.exclusion, self.ei_stop = float(radius0), float(shrink), float(exclusion), ei_stop
        self.gradient, self.line_starts, self.ckpt_every = gradient, int(line_starts), int(ckpt_every)
        self.n_select, self.noise = int(n_select), float(noise)
        self.journal = journal
        # the whole acquisition search on the device (boac_gp_chaos_search); the same proposals as the
        # host loop (chaotic_acquire), so it is not part of the journal's configuration
        self.device_search = bool(device_search)
        self.cycles: List[Cycle] = []
        if journal and os.path.exists(journal):
            self._replay(journal)
        elif journal:
            with open(journal, "w") as f:
                f.write(json.dumps({"config": self._config()}) + "\n")

    # ---- bookkeeping ---------------------------------------------------------------------------
    def _config(self):
        return {"lo": self.lo.tolist(), "hi": self.hi.tolist(), "delta_r": self.delta_r, "n_iter": self.n_iter,
                "n_init": self.n_init, "batch": self.batch, "xi": self.xi, "seed": self.seed,
                "chains": self.chains, "n_global": self.n_global, "n_local": self.n_local, "centres": self.centres,
                "radius0": self.radius0, "shrink": self.shrink, "exclusion": self.exclusion,
                "gradient": self.gradient, "line_starts": self.line_starts, "ckpt_every": self.ckpt_every,
                "n_select": self.n_select, "noise": self.noise,
                "geom": [self.geom.n, self.geom.n_angles, self.geom.n_bins, self.geom.n_samples, self.geom.pixel]}

    def _replay(self, path):
        with open(path) as f:
            lines = [json.loads(l) for l in f if l.strip()]
        if not lines or "config" not in lines[0]:
            raise ValueError(f"{path} is not a BOAC journal")
        if lines[0]["config"] != json.loads(json.dumps(self._config())):
            raise ValueError(f"{path} was written with another configuration")
        self.cycles = [Cycle.from_json(r) for r in lines[1:]]

    def _append(self, cyc: Cycle):
        self.cycles.append(cyc)
        if self.journal:
            with open(self.journal, "a") as f:
                f.write(json.dumps(cyc.to_json()) + "\n")

    def observations(self):
        th = np.concatenate([c.theta for c in self.cycles]) if self.cycles else np.empty((0, 8))
        J = np.concatenate([c.J for c in self.cycles]) if self.cycles else np.empty(0)
        G = None
        if self.gradient and self.cycles:
            G = np.concatenate([c.grad for c in self.cycles])
        return th, J, G

    def best(self):
        th, J, _ = self.observations()
        ok = np.isfinite(J)
        i = int(np.flatnonzero(ok)[np.argmin(J[ok])])
        return th[i], float(J[i])

    def _rng(self, cycle: int, stream: int):
        return np.random.default_rng(np.random.SeedSequence([self.seed, cycle, stream]))

    # ---- evaluation (steps 2-3) ----------------------------------------------------------------
    def _evaluate(self, theta: np.ndarray):
        cand = torch.as_tensor(theta.astype(np.float32), device=self.ctx.device).contiguous()
        if self.gradient:
            J, G, st = self.ctx.objective_grad_ex(self.geom, self.meas, cand, self.delta_r, self.n_iter,
                                                  self.ckpt_every, mode=self.gradient)
            G = G[:, :8].double().cpu().numpy()
        else:
            J, _, st = self.ctx.objective(self.geom, self.meas, cand, self.delta_r, self.n_iter)
            G = None
        return (cand.double().cpu().numpy(), J.double().cpu().numpy(), G, st.cpu().numpy())

    # ---- acquisition (step 5) ------------------------------------------------------------------
    def _acquire(self, model, best: float, cycle: int, q: int, taken: np.ndarray):
        d = self.lo.size
        rng = self._rng(cycle, 1)
        z = rng.uniform(0.01, 0.99, size=(self.chains, d))

        dev = self.ctx.device
        per_step = max(4 * q, 256)
        if self.device_search:
            f64 = torch.float64
            tk = None if taken is None or len(taken) == 0 else torch.tensor(np.asarray(taken, np.float64), dtype=f64,
                                                                           device=dev)
            props, vmax, nq = self.ctx.gp_chaos_search(model, best, self.xi, torch.tensor(z, dtype=f64, device=dev), tk,
                                                      q, n_global=self.n_global, n_local=self.n_local,
                                                      centres=self.centres, radius0=self.radius0, shrink=self.shrink,
                                                      exclusion=self.exclusion, per_step=per_step)
            return props.cpu().numpy(), vmax, nq

        def ei_of(U):
            return self.ctx.gp_ei(model, torch.as_tensor(U, device=dev), best, self.xi).cpu().numpy()

        return chaotic_acquire(ei_of, z, q, taken, n_global=self.n_global, n_local=self.n_local,
                               centres=self.centres, radius0=self.radius0, shrink=self.shrink,
                               exclusion=self.exclusion, per_step=per_step)

    # ---- the loop -------------------------------------------------------------------------------
    def step(self) -> Cycle:
        """Run one cycle (the initial design first) and return it."""
        k = len(self.cycles)
        d = self.lo.size
        t0 = time.perf_counter()
        if k == 0:
            U = self._rng(0, 0).uniform(size=(self.n_init, d))
            theta = self.lo + U * (self.hi - self.lo)
            th, J, G, st = self._evaluate(theta)
            torch.cuda.synchronize()
            cyc = Cycle(0, th, J, G, st, ["init"] * len(J), float("nan"), float("nan"),
                        {"evaluate_ms": 1e3 * (time.perf_counter() - t0)})
            self._append(cyc)
            return cyc
        th_all, J_all, G_all = self.observations()
        ok = np.isfinite(J_all)
        U_all = (th_all[ok] - self.lo) / (self.hi - self.lo)
        model = gp_fit(U_all, J_all[ok], LENGTH_GRID, n_select=self.n_select, noise=self.noise)
        t1 = time.perf_counter()
        best = float(J_all[ok].min())
        q_line = 0
        line_U = np.empty((0, d))
        if self.gradient:
            # line searches along -grad J from the best observations (unit-box gradient: dJ/du = dJ/dtheta (hi - lo))
            order = np.argsort(J_all[ok], kind="stable")[: self.line_starts]
            Gu = G_all[ok] * (self.hi - self.lo)
            kept = []
            for i in order:
                # in order of step length, away from every evaluated point but the start itself and from
                # the line points already kept
                seg = line_search_points(U_all[i], Gu[i])
                if not len(seg):
                    continue
                taken = np.vstack([np.delete(U_all, i, axis=0)] + kept)
                room = self.batch // 2 - sum(len(k) for k in kept)
                pick = greedy_select(seg, -np.arange(len(seg), dtype=np.float64), room, self.exclusion, taken)
                kept.append(seg[sorted(pick)])
            line_U = np.concatenate(kept) if kept else line_U
            q_line = len(line_U)
        newU, max_ei, n_q = self._acquire(model, best, k, self.batch - q_line, np.vstack([U_all, line_U]))
        t2 = time.perf_counter()
        U = np.vstack([newU, line_U])
        theta = self.lo + U * (self.hi - self.lo)
        th, J, G, st = self._evaluate(theta)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        cyc = Cycle(k, th, J, G, st, ["ei"] * len(newU) + ["line"] * len(line_U), max_ei / model.info.s,
                    model.info.length, {"fit_ms": 1e3 * (t1 - t0), "acquire_ms": 1e3 * (t2 - t1),
                                        "evaluate_ms": 1e3 * (t3 - t2), "ei_queries": n_q})
        self._append(cyc)
        return cyc

    def run(self, n_cycles: int):
        """Run until n_cycles cycles (counting the initial design) exist or EI falls below ei_stop."""
        while len(self.cycles) < n_cycles:
            cyc = self.step()
            if self.ei_stop is not None and cyc.index > 0 and cyc.max_ei < self.ei_stop:
                break
        return self.best()


__all__ = ["BOAC", "Cycle", "chaotic_acquire", "greedy_select", "line_search_points", "DEFAULT_LO", "DEFAULT_HI"]
