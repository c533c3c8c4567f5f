"""Continuous-batching solve server over the batch engine (bxmg_batch_*).

Requests (phi, rhs, beta or None, tolerance) wait in a FIFO queue per
coefficient kind and are admitted into that kind's batch as soon as their
device footprint fits in its arena (the library refuses with EBUSY
otherwise).  Every pump() launches a few cycles of both batches -- each on
its own stream, so their work overlaps on the device -- then collects them;
problems that joined while others were mid-solve simply join the next
cycle's launches.  MultiFabs stay on the device throughout.  All the work
runs in libbxmg; this module only orders the calls.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field

from .solver import Batch


@dataclass
class Request:
    tag: object
    phi: object
    rhs: object
    beta: object = None
    rel_tol: float = 0.0
    t_submit: float = field(default_factory=time.perf_counter)


class Server:
    """Server(ctx, budget_bytes, max_problems=256, chunk=1, var_share=0.5,
    **solve params).  var_share: fraction of the budget for the batch of
    variable-coefficient problems."""

    def __init__(self, ctx, budget_bytes, max_problems=256, chunk=1, var_share=0.5, **params):
        self.chunk = int(chunk)
        vb = int(budget_bytes * var_share)
        self.batches = {}
        if budget_bytes - vb > 0:
            self.batches[False] = Batch(ctx, budget_bytes - vb, max_problems, var=False, **params)
        if vb > 0:
            self.batches[True] = Batch(ctx, vb, max_problems, var=True, **params)
        self.queues = {False: deque(), True: deque()}
        self.live = {}  # (kind, id) -> Request
        self.rejected = []

    def close(self):
        for b in self.batches.values():
            b.close()

    def submit(self, tag, phi, rhs, beta=None, rel_tol=0.0):
        self.queues[beta is not None].append(Request(tag, phi, rhs, beta, rel_tol))

    def pending(self):
        return sum(len(q) for q in self.queues.values())

    def running(self):
        return len(self.live)

    def idle(self):
        return not self.live and self.pending() == 0

    def _admit(self):
        for kind, q in self.queues.items():
            b = self.batches.get(kind)
            while q and b is None:  # no storage for this kind at all
                self.rejected.append((q.popleft().tag, "no batch for this coefficient kind"))
            while q:
                r = q[0]
                try:
                    pid = b.add(r.phi, r.rhs, r.beta, r.rel_tol)
                except Exception as e:  # cannot run in a batch at all
                    q.popleft()
                    self.rejected.append((r.tag, str(e)))
                    continue
                if pid is None:
                    break
                q.popleft()
                self.live[(kind, pid)] = r

    def pump(self):
        """Admit what fits, run `chunk` cycles of every busy batch, and return
        the requests that finished: [(tag, SolveResult, t_done)]."""
        self._admit()
        busy = [k for k in self.batches if any(key[0] == k for key in self.live)]
        for k in busy:
            self.batches[k].launch(self.chunk)
        for k in busy:
            self.batches[k].collect()
        out = []
        now = time.perf_counter()
        for k, b in self.batches.items():
            for pid, res in b.poll():
                r = self.live.pop((k, pid))
                out.append((r.tag, res, now))
        return out
