"""Continuous-batching solve server over resident QTT operators.

Each operator is a pair (A, Ainv) of QTT matrices held on the device for the
server's lifetime: A in FP64 for the residual, Ainv in a low-precision dtype
for the refinement.  Requests (an operator id and a block of right-hand
sides) arrive over time.  A fixed number of slots, each a host thread with
its own HIP stream, run refined solves (``qtt_solve``) concurrently, so work
of different batches overlaps on the device.  Whenever a slot is free, the
scheduler admits the oldest waiting request's operator and coalesces every
waiting request for that operator into one batch, as far as the device
memory budget and the batch width allow; requests that arrive while other
batches run are admitted as soon as a slot and memory free up.

The per-column arithmetic of the apply and of the solve does not depend on
the other columns of a batch (no cross-column reductions, a fixed kernel per
core once an operator is loaded), so a request's result is the same alone
and in any mix.

All numerics run in libqtt; this module only schedules, copies request
blocks into batch buffers, and records latencies.
"""
from __future__ import annotations

import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import qtt as Q


@dataclass
class Request:
    rid: int
    op: str
    F: torch.Tensor               # (N, k) column-major FP64 on the device
    arrival: float = 0.0          # seconds on the server clock
    Sigma: torch.Tensor | None = None
    info: list = field(default_factory=list)
    status: int = -1
    admitted: float = -1.0
    done: float = -1.0
    batch_id: int = -1
    error: str = ""

    @property
    def k(self):
        return 1 if self.F.dim() == 1 else self.F.shape[1]

    @property
    def latency(self):
        return self.done - self.arrival


class Arena:
    """First-fit sub-allocator over one device buffer of the whole budget.

    The server's batches take their workspace, right-hand sides and solutions
    from here, so the budget is the memory actually reserved (no caching
    allocator fragmentation can make an admitted batch fail)."""

    ALIGN = 256

    def __init__(self, nbytes, device):
        self.size = int(nbytes) // self.ALIGN * self.ALIGN
        self.buf = torch.empty(self.size, dtype=torch.uint8, device=device)
        self.free = [(0, self.size)]          # sorted (offset, length)

    def alloc(self, nbytes):
        n = (int(nbytes) + self.ALIGN - 1) // self.ALIGN * self.ALIGN
        for i, (off, ln) in enumerate(self.free):
            if ln >= n:
                if ln == n:
                    self.free.pop(i)
                else:
                    self.free[i] = (off + n, ln - n)
                return off, n
        return None

    def release(self, off, n):
        self.free.append((off, n))
        self.free.sort()
        merged = []
        for o, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == o:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((o, ln))
        self.free = merged

    def largest(self):
        return max((ln for _, ln in self.free), default=0)

    def block(self, off, N, k):
        """(N, k) FP64 column-major view at byte offset off."""
        return self.buf[off:off + N * k * 8].view(torch.float64).view(k, N).t()

    def bytes(self, off, n):
        return self.buf[off:off + n]


def choose_batch(pending, in_use, budget, max_rhs, bytes_fn):
    """Admission policy.  pending: {op: deque of requests in arrival order}
    (each with .arrival and .k).  Operators are tried in the order of their
    oldest waiting request; for the first one whose oldest request fits the
    remaining budget, the waiting requests are taken in arrival order while
    the batch stays within max_rhs columns and the budget.  Returns
    (op, requests, columns, bytes) or None when nothing fits now."""
    heads = sorted((q[0].arrival, op) for op, q in pending.items() if q)
    for _, op in heads:
        reqs, k = [], 0
        for r in pending[op]:
            if reqs and k + r.k > max_rhs:
                break
            if in_use + bytes_fn(op, k + r.k) > budget:
                break
            reqs.append(r)
            k += r.k
        if reqs:
            return op, reqs, k, bytes_fn(op, k)
    return None


class SolveServer:
    """Refined solves for resident operators with continuous batching.

    operators: {name: (A_cores, Ainv_cores)} host FP64 cores.
    budget_bytes: device memory the batches in flight may hold together
        (solve workspace + batch right-hand sides + solutions).
    residual_lo, lo_below: with a dtype ("fp32"), each operator also keeps
        a copy of A in it, and a request column that starts a refinement
        pass at or below lo_below of its right-hand side's norm updates its
        residual with that copy (r -= A_lo dx, qtt_solve_schedule) instead
        of recomputing it in FP64; choose lo_below <= 0.01 rtol / u_lo.
    """

    def __init__(self, operators, inv_dtype="bf16", budget_bytes=200 * 10 ** 9, n_slots=3,
                 rtol=1e-8, max_iter=50, max_batch_rhs=64, device="cuda", residual_lo=None, lo_below=0.0):
        self.inv_dtype = inv_dtype
        self.residual_lo = residual_lo
        self.lo_below = float(lo_below)
        self.budget = int(budget_bytes)
        self.rtol = rtol
        self.max_iter = max_iter
        self.max_batch_rhs = max_batch_rhs
        self.device = torch.device(device)
        self.ops = {}
        self.lo = {}
        for name, (Ac, Aic) in operators.items():
            A = Q.qtt_matrix_load(Ac, dtypes=("fp64",))
            Ai = Q.qtt_matrix_load(Aic, dtypes=(inv_dtype,))
            self.ops[name] = (A, Ai)
            if residual_lo is not None:
                self.lo[name] = Q.qtt_matrix_load(Ac, dtypes=(residual_lo,))
        self.n_slots = n_slots
        self.arena = Arena(self.budget, self.device)
        self._lock = threading.Condition()
        self._pending = {name: deque() for name in self.ops}
        self._in_use = 0
        self._busy = 0
        self._closed = False
        self._batches = 0
        self.t0 = time.perf_counter()
        self.log = []                 # (batch_id, op, rids, admitted, done)
        self._workers = [threading.Thread(target=self._worker, args=(i,), daemon=True)
                         for i in range(n_slots)]
        for w in self._workers:
            w.start()

    # ------------------------------------------------------------ memory model
    def batch_bytes(self, op, k):
        return self._arena_bytes(op, k)

    def now(self):
        return time.perf_counter() - self.t0

    # ------------------------------------------------------------ client side
    def submit(self, req: Request):
        if req.op not in self.ops:
            raise KeyError(f"unknown operator {req.op}")
        A, _ = self.ops[req.op]
        if req.F.shape[0] != A.rows:
            raise ValueError("right-hand side length does not match the operator")
        if self.batch_bytes(req.op, req.k) > self.budget:
            raise MemoryError(f"request {req.rid} needs more than the whole budget")
        with self._lock:
            req.arrival = self.now() if req.arrival <= 0 else req.arrival
            self._pending[req.op].append(req)
            self._lock.notify_all()

    def close(self):
        with self._lock:
            self._closed = True
            self._lock.notify_all()
        for w in self._workers:
            w.join()
        for A, Ai in self.ops.values():
            A.free()
            Ai.free()
        for A_lo in self.lo.values():
            A_lo.free()
        self.arena = None            # the budget's device memory goes back to torch

    # ------------------------------------------------------------ scheduling
    def _take_batch(self):
        """Called with the lock held: the next batch, or None."""
        # the budget seen by the policy is the largest free block of the arena
        free = self.arena.largest()
        got = choose_batch(self._pending, self.budget - free, self.budget, self.max_batch_rhs,
                           self._arena_bytes)
        if got is None:
            return None
        op, reqs, k, _ = got
        region = self.arena.alloc(self._arena_bytes(op, k))
        if region is None:
            return None
        for _ in reqs:
            self._pending[op].popleft()
        self._in_use += region[1]
        self._batches += 1
        return op, reqs, k, region, self._batches

    def _arena_bytes(self, op, k):
        """Bytes of one batch as carved from the arena (each part aligned)."""
        A, Ai = self.ops[op]
        al = Arena.ALIGN
        ws = Q.qtt_solve_schedule_workspace_bytes(A, Ai, self.inv_dtype, k, **self._schedule(op))
        blk = (A.rows * k * 8 + al - 1) // al * al
        return (ws + al - 1) // al * al + 2 * blk

    def _schedule(self, op):
        if self.residual_lo is None:
            return {}
        return dict(A_lo=self.lo[op], lo_compute=self.residual_lo, lo_below=self.lo_below)

    def _worker(self, slot):
        stream = torch.cuda.Stream(device=self.device)
        while True:
            with self._lock:
                while True:
                    if self._closed and not any(self._pending.values()):
                        return
                    got = self._take_batch()
                    if got is not None:
                        break
                    self._lock.wait(timeout=0.05)
                self._busy += 1
            op, reqs, k, region, bid = got
            t_adm = self.now()
            try:
                self._run(op, reqs, k, stream, bid, t_adm, region)
            except Exception as e:          # report the failure on the requests, keep serving
                t = self.now()
                for r in reqs:
                    r.status, r.done, r.admitted, r.batch_id = -2, t, t_adm, bid
                    r.error = repr(e)
            finally:
                # nothing queued on the slot stream may still use the region
                # when it goes back to the arena (also after a failed batch)
                try:
                    stream.synchronize()
                except Exception:
                    pass
                with self._lock:
                    self.arena.release(*region)
                    self._in_use -= region[1]
                    self._busy -= 1
                    self._lock.notify_all()

    def _run(self, op, reqs, k, stream, bid, t_adm, region):
        A, Ai = self.ops[op]
        N = A.rows
        al = Arena.ALIGN
        off0, _ = region
        ws_n = (Q.qtt_solve_schedule_workspace_bytes(A, Ai, self.inv_dtype, k, **self._schedule(op))
                + al - 1) // al * al
        blk = (N * k * 8 + al - 1) // al * al
        ws = self.arena.bytes(off0, ws_n)
        Fb = self.arena.block(off0 + ws_n, N, k)
        Sb = self.arena.block(off0 + ws_n + blk, N, k)
        stream.wait_stream(torch.cuda.default_stream(self.device))   # request blocks are ready
        with torch.cuda.stream(stream):
            c = 0
            for r in reqs:
                Fb[:, c:c + r.k].copy_(r.F.reshape(N, r.k))
                c += r.k
        _, info, st = Q.qtt_solve_schedule(A, Ai, self.inv_dtype, Fb, Sb, rtol=self.rtol, max_iter=self.max_iter,
                                           ws=ws, stream=stream, raise_on_fail=False, **self._schedule(op))
        with torch.cuda.stream(stream):
            outs = []
            c = 0
            for r in reqs:        # results leave the arena before the region is reused
                o = Q.empty_block(N, r.k, self.device)
                o.copy_(Sb[:, c:c + r.k])
                outs.append(o)
                c += r.k
        stream.synchronize()
        t_done = self.now()
        c = 0
        for r, o in zip(reqs, outs):
            r.Sigma = o
            r.info = info[c:c + r.k]
            r.status = st
            r.admitted = t_adm
            r.done = t_done
            r.batch_id = bid
            c += r.k
        with self._lock:
            self.log.append((bid, op, [r.rid for r in reqs], t_adm, t_done))

    # ------------------------------------------------------------ traces
    def run_trace(self, requests, realtime=True):
        """Submit requests at their arrival times (seconds from now), wait for
        all of them, and return summary statistics."""
        start = self.now()
        for r in sorted(requests, key=lambda r: r.arrival):
            if realtime:
                delay = start + r.arrival - self.now()
                if delay > 0:
                    time.sleep(delay)
            r.arrival = start + r.arrival
            self.submit(r)
        while True:
            with self._lock:
                if all(r.done >= 0 for r in requests):
                    break
                self._lock.wait(timeout=0.05)
        return summarize(requests)


def summarize(requests):
    lat = np.array([r.latency for r in requests]) * 1e3
    rhs = sum(r.k for r in requests)
    t_first = min(r.arrival for r in requests)
    t_last = max(r.done for r in requests)
    worst = max((c[1] for r in requests for c in r.info), default=float("nan"))
    return {"requests": len(requests), "rhs": rhs, "wall_s": t_last - t_first,
            "rhs_per_s": rhs / (t_last - t_first), "p50_ms": float(np.percentile(lat, 50)),
            "p99_ms": float(np.percentile(lat, 99)), "max_rel_residual": worst,
            "batches": len({r.batch_id for r in requests}),
            "all_converged": all(r.status == 0 for r in requests),
            "status_counts": {str(s): sum(1 for r in requests if r.status == s)
                              for s in sorted({r.status for r in requests})},
            "first_error": next((r.error for r in requests if r.error), ""),
            "iters_max": max((c[0] for r in requests for c in r.info), default=0)}


def serving_operators(n_ops=12, levels=(5, 6, 7, 8), seed=51):
    """The serving workload's resident operators: {name: (A_cores, Ainv_cores)}
    and their descriptions (L, ranks)."""
    from . import inputs as I
    descs = I.serving_operators(n_ops, levels=levels, seed=seed)
    operators = {}
    for t, dsc in enumerate(descs):
        A, Ai = I.perturbed_identity_pair(dsc["ranks"], [8] * dsc["L"], seed=dsc["seed"], eps=0.1)
        operators[f"op{t}"] = (A, Ai)
    return operators, descs


def serving_trace(server, descs, n_requests, rate, seed=51, k_max=16, device="cuda"):
    """Run a seeded Poisson trace on a server: request i picks an operator and
    k in [1, k_max] from a seeded generator; its right-hand sides are drawn
    N(0,1) on the device from a seeded torch generator.  Returns the summary
    of summarize(), plus per-L latency percentiles and the largest relative
    residual ||F - A Sigma|| / ||F|| recomputed by a separate FP64 apply."""
    from . import inputs as I
    g = I.rng(seed + 1)
    arrivals = I.poisson_arrivals(n_requests, rate, seed=seed + 2)
    tg = torch.Generator(device=device).manual_seed(seed * 7919)
    reqs = []
    for i in range(n_requests):
        t = int(g.integers(len(descs)))
        k = int(g.integers(1, k_max + 1))
        N = 8 ** descs[t]["L"]
        F = torch.randn((k, N), generator=tg, device=device, dtype=torch.float64).t()
        reqs.append(Request(rid=i, op=f"op{t}", F=F, arrival=float(arrivals[i])))
    torch.cuda.synchronize()
    stats = server.run_trace(reqs)
    by_L = {}
    for r in reqs:
        by_L.setdefault(descs[int(r.op[2:])]["L"], []).append(r.latency * 1e3)
    stats["latency_by_L_ms"] = {str(L): {"requests": len(v), "p50": float(np.percentile(v, 50)),
                                         "p99": float(np.percentile(v, 99))}
                                for L, v in sorted(by_L.items())}
    worst = 0.0
    # one workspace of the one-vector size of the largest operator: the
    # recomputation runs in waves of single vectors beside the arena
    ws = Q.workspace(max(Q.qtt_workspace_bytes(A, "fp64", 1) for A, _ in server.ops.values()), device)
    for r in reqs:
        if r.Sigma is None:
            continue
        A, _ = server.ops[r.op]
        AS = Q.qtt_apply(A, "fp64", r.Sigma.reshape(A.rows, -1), ws=ws)
        res = (r.F.reshape(A.rows, -1) - AS).norm(dim=0) / r.F.reshape(A.rows, -1).norm(dim=0)
        worst = max(worst, float(res.max()))
        r.Sigma = None
    stats["max_rel_residual_recomputed"] = worst
    return stats


def _main():
    """Serving benchmark: a seeded Poisson trace over resident operators."""
    import argparse
    import json
    p = argparse.ArgumentParser()
    p.add_argument("--requests", type=int, default=48)
    p.add_argument("--rate", type=float, default=200.0)
    p.add_argument("--ops", type=int, default=12)
    p.add_argument("--levels", default="5,6,7,8")
    p.add_argument("--slots", type=int, default=3)
    p.add_argument("--inv", default="bf16")
    p.add_argument("--budget-gb", type=float, default=200.0)
    p.add_argument("--seed", type=int, default=51)
    args = p.parse_args()
    levels = tuple(int(x) for x in args.levels.split(","))
    operators, descs = serving_operators(args.ops, levels=levels, seed=args.seed)
    srv = SolveServer(operators, inv_dtype=args.inv, budget_bytes=int(args.budget_gb * 1e9),
                      n_slots=args.slots)
    stats = serving_trace(srv, descs, args.requests, args.rate, seed=args.seed)
    srv.close()
    stats.update({"workload": "serving: Poisson trace over resident QTT operators",
                  "operators": [{"L": d["L"], "r": d["ranks"][1]} for d in descs],
                  "rate_per_s": args.rate, "slots": args.slots, "inverse_dtype": args.inv,
                  "budget_gb": args.budget_gb})
    print(json.dumps(stats), flush=True)


if __name__ == "__main__":
    _main()
