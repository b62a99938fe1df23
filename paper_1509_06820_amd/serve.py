"""A continuous-batching server of truncated-SVD requests (TUXV, Alg. 7 with
j_max = 1 and the SVD of X) on one GPU.

Requests arrive over time, each a device-resident matrix with its rank k and
precision.  The server admits them while their HBM footprint (matrix,
outputs and the workspace the library asks for) fits a budget, and launches
work as soon as a stream of its pool is free:

* requests with k <= 64 go to the batched engine (rq_batch_plan_create /
  rq_tuxv_batched): every admitted, not yet started request of the same
  (k, precision) joins one batch, in arrival order;
* larger ranks run the single-matrix path (rq_tuxv) on their own stream.

Batches and single solves of different streams overlap on the device; new
requests are admitted and launched while earlier ones run (continuous
batching, not a queue drained batch by batch).  Completion is observed by
polling events, latency is arrival -> completion as the host sees it.  The
result of a request does not depend on the other requests it is batched
with (each matrix's work touches only its own buffers), which the tests
check bit for bit.
"""

import time
from collections import deque

import numpy as np
import torch

from . import binding

BATCH_KMAX = 64


class Request:
    def __init__(self, rid, A, k, precision, seed, arrival):
        self.id = rid
        self.A = binding.fortran(A)
        self.k = int(k)
        self.precision = binding._prec(precision)
        self.seed = int(seed)
        self.arrival = float(arrival)
        self.t_admit = None
        self.t_done = None
        self.U = self.sigma = self.VT = None
        self.info = None
        self.engine = None

    @property
    def batched(self):
        m, n = self.A.shape
        return self.k <= BATCH_KMAX and n <= 8192 and self.precision != binding.RQ_MIXED_BF16


def block_size(k, batched):
    """b for a request: the largest power of two <= 32 dividing k (batched;
    b + p <= 64), 64 or k (single path)."""
    if not batched:
        return min(64, k)
    b = 32
    while b > 1 and k % b:
        b //= 2
    return b


class TuxvServer:
    def __init__(self, hbm_budget, streams=4, p=8, max_batch=128, poll_sleep=20e-6):
        self.budget = float(hbm_budget)
        self.p = p
        self.max_batch = max_batch
        self.poll_sleep = poll_sleep
        self.streams = [torch.cuda.Stream() for _ in range(streams)]
        self.busy = [None] * streams   # the unit in flight on each stream
        self.used = 0.0
        self.max_used = 0.0

    # footprint of one request (bytes): its workspace share and its outputs
    def footprint(self, r):
        m, n = r.A.shape
        b = block_size(r.k, r.batched)
        if r.batched:
            ws = binding.batch_workspace_bytes([(m, n)], r.k, b, self.p, r.precision)
        else:
            ws = binding.rq_workspace_bytes(binding.RQ_OP_TUXV, m, n, r.k, b, self.p, r.precision)
        return ws + 8.0 * (m * r.k + r.k * n + r.k)

    def _launch(self, si, reqs, now):
        s = self.streams[si]
        with torch.cuda.stream(s):
            if reqs[0].batched:
                r0 = reqs[0]
                b = block_size(r0.k, True)
                bt = binding.BatchTUXV([r.A for r in reqs], r0.k, b, self.p, [r.seed for r in reqs],
                                       precision=r0.precision)
                bt.run(stream=s)
                for i, r in enumerate(reqs):
                    r.U, r.sigma, r.VT, r.info = bt.U[i], bt.sigma[i], bt.VT[i], bt.info[i:i + 1]
                    r.engine = "batched"
                keep = bt
            else:
                r = reqs[0]
                b = block_size(r.k, False)
                r.U, r.sigma, r.VT, r.info = binding.rq_tuxv(r.A, r.k, b, self.p, r.seed, stream=s,
                                                             precision=r.precision)
                r.engine = "single"
                keep = None
            ev = torch.cuda.Event()
            ev.record(s)
        for r in reqs:
            r.t_admit = now
        self.busy[si] = dict(reqs=reqs, event=ev, keep=keep, bytes=sum(r._fp for r in reqs))

    def serve(self, requests, clock=time.perf_counter):
        """Serve `requests` (sorted by arrival, seconds from the start).
        Returns a dict of statistics; each request gets its outputs and its
        admission and completion times."""
        pending = deque()
        arrivals = deque(sorted(requests, key=lambda r: r.arrival))
        done = []
        for r in requests:
            r._fp = self.footprint(r)
            if r._fp > self.budget:
                raise ValueError(f"request {r.id} needs {r._fp:.3g} bytes, more than the budget")
        t0 = clock()
        n_total = len(requests)
        while len(done) < n_total:
            now = clock() - t0
            while arrivals and arrivals[0].arrival <= now:
                pending.append(arrivals.popleft())
            progressed = False
            # completions
            for si, unit in enumerate(self.busy):
                if unit is not None and unit["event"].query():
                    t = clock() - t0
                    for r in unit["reqs"]:
                        r.t_done = t
                        done.append(r)
                    self.used -= unit["bytes"]
                    unit["keep"] = None
                    self.busy[si] = None
                    progressed = True
            # admission and launch on free streams
            while pending:
                free = [si for si, u in enumerate(self.busy) if u is None]
                if not free:
                    break
                head = pending[0]
                if self.used + head._fp > self.budget:
                    break
                if head.batched:
                    group, rest, fp = [], deque(), 0.0
                    for r in pending:
                        if (len(group) < self.max_batch and r.batched and r.k == head.k
                                and r.precision == head.precision and self.used + fp + r._fp <= self.budget):
                            group.append(r)
                            fp += r._fp
                        else:
                            rest.append(r)
                    pending = rest
                else:
                    group = [pending.popleft()]
                    fp = head._fp
                self.used += fp
                self.max_used = max(self.max_used, self.used)
                self._launch(free[0], group, now)
                progressed = True
            if not progressed:
                if arrivals and not pending and all(u is None for u in self.busy):
                    wait = arrivals[0].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 1e-3))
                else:
                    time.sleep(self.poll_sleep)
        torch.cuda.synchronize()
        lat = np.array([r.t_done - r.arrival for r in requests])
        span = max(r.t_done for r in requests) - min(r.arrival for r in requests)
        out = {"requests": n_total, "span_s": span, "solves_per_s": n_total / span if span > 0 else None,
               "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "mean_ms": float(lat.mean() * 1e3), "max_hbm_bytes": self.max_used,
               "batched": sum(r.engine == "batched" for r in requests),
               "single": sum(r.engine == "single" for r in requests)}
        for prec in sorted({r.precision for r in requests}):
            lp = np.array([r.t_done - r.arrival for r in requests if r.precision == prec])
            out[f"p50_ms_prec{prec}"] = float(np.percentile(lp, 50) * 1e3)
            out[f"p99_ms_prec{prec}"] = float(np.percentile(lp, 99) * 1e3)
        return out


def serving_matrix_device(i, m, n, seed=5, device="cuda"):
    """The matrix of served request i made on the GPU: U diag(0.95^j) V^T with
    Haar factors (QR of Gaussians, sign-fixed) drawn from a torch generator
    seeded with seed * 100003 + i; triplets below 1e-17 sigma_0 dropped."""
    g = torch.Generator(device=device)
    g.manual_seed(seed * 100003 + i)
    q = min(m, n)
    r = min(q, int(np.ceil(np.log(1e-17) / np.log(0.95))))

    def haar(rows):
        G = torch.randn(rows, r, generator=g, dtype=torch.float64, device=device)
        Q, R = torch.linalg.qr(G)
        d = torch.sign(torch.diagonal(R))
        d[d == 0] = 1.0
        return Q * d

    U = haar(m)
    V = haar(n)
    sig = 0.95 ** torch.arange(r, dtype=torch.float64, device=device)
    A = (U * sig) @ V.T
    return A.t().contiguous().t()
