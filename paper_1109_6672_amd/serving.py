"""Request loop over the continuous-batching server, and the one-solve-at-a-time
baseline it is compared with (same kernels, one grid per launch, first in
first out).  Both report per-request time-to-finish from the arrival time,
p50/p99 latency, solves per second and aggregate MLUPS."""
from __future__ import annotations

import sys
import time

import numpy as np

from . import lbddf, workloads as W


def _pct(v, q):
    return float(np.percentile(np.array(v), q)) if v else None


def _summary(lat, node_updates, wall, states, steps, edges):
    """p50/p99 of the time from arrival to finish over every request, and
    over the requests that reached a steady state (converged or plateau):
    their time-to-converged; steps per request by outcome (median); outcomes
    per grid edge."""
    done = [t for t, s in zip(lat, states) if s in ("converged", "plateau")]
    by, per_edge = {}, {}
    for s, n, e in zip(states, steps, edges):
        by.setdefault(s, []).append(n)
        d = per_edge.setdefault(str(e), {})
        d[s] = d.get(s, 0) + 1
    return dict(n=len(states), p50_s=_pct(lat, 50), p99_s=_pct(lat, 99),
                converged_p50_s=_pct(done, 50), converged_p99_s=_pct(done, 99),
                solves_per_s=len(states) / wall, mlups=node_updates / wall / 1e6, wall_s=wall,
                states={s: states.count(s) for s in sorted(set(states))},
                median_steps={s: int(np.median(v)) for s, v in sorted(by.items())},
                states_by_edge=per_edge)


class Plateau:
    """The server's plateau test (lbs_advance): the residual lies below 1e-2
    of its largest value so far and has made no new minimum for max(10, n/2)
    of the n checks so far, minima counted from that maximum."""

    def __init__(self):
        self.peak, self.best, self.stall, self.checks = 0.0, np.inf, 0, 0

    def update(self, r: float) -> bool:
        self.checks += 1
        if r > self.peak:
            self.peak = self.best = r
            self.stall = 0
        elif r < self.best:
            self.best, self.stall = r, 0
        else:
            self.stall += 1
            if self.stall >= max(10, self.checks // 2) and r < 1e-2 * self.peak:
                return True
        return False


def _report(every, last, now, label, done, total, extra=""):
    """A progress line on stderr at most every `every` seconds (0: never)."""
    if every and now - last >= every:
        print(f"[serving] {label}: {done}/{total} finished after {now:.0f} s{extra}", file=sys.stderr, flush=True)
        return now
    return last


def run_server(requests, pool_bytes, storage="f32", k_steps=200, tol=1e-6, max_steps=20000, realtime=True,
               progress=0.0):
    """Drives a Server with the requests' arrival times (seconds from start);
    progress > 0 prints a line on stderr every that many seconds."""
    srv = lbddf.Server(pool_bytes, storage=storage, k_steps=k_steps)
    pending = sorted(requests, key=lambda r: r["t"])
    ids, i = {}, 0
    t0 = time.perf_counter()
    last = 0.0
    while True:
        live = sum(srv.poll(rid)["state"] in ("queued", "running") for rid in ids)
        if i >= len(pending) and live == 0:
            break
        now = time.perf_counter() - t0
        last = _report(progress, last, now, f"packed {storage}", len(ids) - live, len(pending))
        while i < len(pending) and (pending[i]["t"] <= now or not realtime):
            r = pending[i]
            ids[srv.submit(r["params"], r.get("fields"), tol=tol, max_steps=max_steps)] = r
            i += 1
        resident, queued = srv.advance()
        if resident == 0 and queued == 0 and i < len(pending):
            time.sleep(max(0.0, min(0.01, pending[i]["t"] - (time.perf_counter() - t0))))
    wall = time.perf_counter() - t0
    lat, states, nodes, steps = [], [], 0.0, []
    for rid, r in ids.items():
        p = srv.poll(rid)
        lat.append(p["t_done"] - (r["t"] if realtime else p["t_submit"]))
        states.append(p["state"])
        steps.append(p["steps"])
        nodes += r["params"]["nx"] * r["params"]["ny"] * p["steps"]
    out = _summary(lat, nodes, wall, states, steps, [r["params"]["nx"] for r in ids.values()])
    out["server"] = srv.stats()
    return out, srv, ids


def run_sequential(requests, storage="f32", k_steps=200, tol=1e-6, max_steps=20000, realtime=True,
                   progress=0.0):
    """One solve at a time, first in first out, one grid per launch: lb_step
    (k steps as replays of its captured graph) and one FP64 residual per
    check, which also reports an unstable grid."""
    pending = sorted(requests, key=lambda r: r["t"])
    t0 = time.perf_counter()
    lat, states, nodes, steps = [], [], 0.0, []
    last = 0.0
    for r in pending:
        now = time.perf_counter() - t0
        last = _report(progress, last, now, f"one at a time {storage}", len(states), len(pending))
        if realtime and r["t"] > now:
            time.sleep(r["t"] - now)
        p = dict(r["params"], storage=storage)
        s = lbddf.Solver(p)
        f = r.get("fields")
        s.init(*(f if f is not None else (None,) * 4))
        s.residual(update=True)
        pl, state = Plateau(), "step_cap"
        while s.time < max_steps:
            s.step(k_steps)
            try:
                res = s.residual(update=True)
            except lbddf.LBError as e:
                if e.status != lbddf.LB_EUNSTABLE:
                    raise
                state = "unstable"
                break
            if res < tol:
                state = "converged"
                break
            if pl.update(res):
                state = "plateau"
                break
        s.macros()
        done = time.perf_counter() - t0
        lat.append(done - (r["t"] if realtime else 0.0))
        states.append(state)
        steps.append(s.time)
        nodes += p["nx"] * p["ny"] * s.time
        s.close()
    wall = time.perf_counter() - t0
    return _summary(lat, nodes, wall, states, steps, [r["params"]["nx"] for r in pending])


def mix(n_requests=32, sizes=(64, 128, 256), rate=50.0, storage="f32"):
    return W.serving_mix(n_requests, sizes=sizes, rate=rate, storage=storage)
