"""Continuous-batching request loop over resident databases.

Requests (each 1..Q encrypted queries against one resident database) are
admitted as launch slots and device memory free up: the loop keeps a queue
per database, and whenever a slot is free it packs the oldest queued queries
of one database into a single batched sanns_distances call on its own HIP
stream, up to a query cap and within the HBM budget.  Launches of different
batches overlap on the device; completion is polled with events, so requests
that arrive while others run are admitted as soon as resources allow.

A linear-scan request needs one server launch; a clustered request needs
two (centre distances, then -- after the client's cleartext cluster choice --
the selected clusters' chunks and the stash), each queued and batched the
same way.  Masks are keyed by (database key, query id, chunk), never by the
batch, so every query's outputs are bit-identical alone and in any mix.

Latency is measured from a request's arrival to the moment its shares are
ready on the device.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, Dict, List, Optional, Sequence

import numpy as np
import torch

from . import clustered as clus
from . import native as nat
from . import stage


@dataclasses.dataclass
class ResidentDB:
    name: str
    ctx: stage.Context
    db: Optional[stage.Database] = None                 # linear-scan database
    server: Optional[clus.ClusteredServer] = None       # clustered index
    key: bytes = b""
    u: int = 64                                         # clusters per query

    @property
    def clustered(self) -> bool:
        return self.server is not None


@dataclasses.dataclass
class Request:
    rid: int
    db: str
    ct: torch.Tensor            # [Q][d][2][L][N] query ciphertexts (device)
    qids: np.ndarray            # [Q] uint64 query ids, unique over the run
    k: int
    arrival: float = 0.0        # seconds since the loop started
    # filled in by the loop
    phase: int = 0              # clustered: 1 = centres done, waiting for phase 2
    selected: Optional[List[np.ndarray]] = None
    outputs: Dict[str, tuple] = dataclasses.field(default_factory=dict)
    done: float = -1.0

    @property
    def Q(self) -> int:
        return int(self.ct.shape[0])


@dataclasses.dataclass
class _Job:
    req: Request
    stage: str                  # "scan", "centres" or "points"


@dataclasses.dataclass
class _Launch:
    slot: int
    jobs: List[_Job]
    dbname: str
    stage: str
    bytes: int
    event: torch.cuda.Event
    stream: torch.cuda.Stream
    out: torch.Tensor
    share: torch.Tensor
    work: Optional[np.ndarray]
    keep: list


class AdmissionError(RuntimeError):
    pass


class Server:
    def __init__(self, dbs: Sequence[ResidentDB], hbm_budget: int, max_inflight: int = 3,
                 max_batch_queries: int = 64, mode: int = nat.SANNS_MODE_FUSED,
                 client_select: Optional[Callable] = None, keep_outputs: bool = True):
        """keep_outputs=False releases each request's output buffers when it
        completes (as a server does once the shares have been sent)."""
        self.dbs = {d.name: d for d in dbs}
        self.hbm_budget = int(hbm_budget)
        self.max_inflight = max_inflight
        self.max_batch_queries = max_batch_queries
        self.mode = mode
        self.client_select = client_select
        self.queues: Dict[tuple, collections.deque] = collections.defaultdict(collections.deque)
        self.inflight: List[_Launch] = []
        self.keep_outputs = keep_outputs
        self.streams = [torch.cuda.Stream() for _ in range(max_inflight)]
        # per launch slot: reusable workspace, query staging and (when outputs
        # are released at completion) output buffers, grown geometrically so
        # that steady-state serving allocates nothing
        self.pool_ws: List[Optional[torch.Tensor]] = [None] * max_inflight
        self.pool_ct: List[Optional[torch.Tensor]] = [None] * max_inflight
        self.pool_out: List[Optional[torch.Tensor]] = [None] * max_inflight
        self.pool_share: List[Optional[torch.Tensor]] = [None] * max_inflight
        self.busy = [False] * max_inflight
        self.used = 0
        self.peak_used = 0
        self.launches = 0
        self.completed: List[Request] = []
        self.t0 = time.perf_counter()

    # ------------------------------------------------------------ footprint
    def _footprint(self, dbname: str, st: str, Q: int, M: int) -> int:
        R = self.dbs[dbname]
        ctx = R.ctx
        if st == "centres":
            desc = R.server.cdb.desc
        elif st == "points":
            desc = R.server.db.desc
        else:
            desc = R.db.desc
        ws = nat.sanns_distances_workspace(ctx.handle, desc, Q, M, self.mode)
        return ws + M * (2 * ctx.L * ctx.N * 8 + ctx.N * 4)

    def _n_chunks(self, dbname: str, st: str) -> int:
        R = self.dbs[dbname]
        if st == "centres":
            return R.server.cdb.n_chunks
        if st == "points":
            return R.server.db.n_chunks
        return R.db.n_chunks

    def _job_M(self, job: _Job) -> int:
        if job.stage == "points":
            return len(self.dbs[job.req.db].server.work_list(job.req.selected))
        return job.req.Q * self._n_chunks(job.req.db, job.stage)

    # ------------------------------------------------------------ interface
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        R = self.dbs[req.db]
        st = "centres" if R.clustered else "scan"
        job = _Job(req, st)
        need = self._footprint(req.db, st, req.Q, self._job_M(job))
        if need > self.hbm_budget:
            raise AdmissionError(f"request {req.rid} needs {need} B > budget {self.hbm_budget} B")
        self.queues[(req.db, st)].append(job)

    def pending(self) -> bool:
        return bool(self.inflight) or any(self.queues.values())

    def poll(self):
        """Retire finished launches, then admit queued work."""
        still = []
        for lx in self.inflight:
            if lx.event.query():
                self._retire(lx)
            else:
                still.append(lx)
        self.inflight = still
        self._admit()

    def run(self, requests: Sequence[Request], realtime: bool = True) -> List[Request]:
        """Serve requests whose `arrival` times are seconds after the start."""
        order = sorted(requests, key=lambda r: r.arrival)
        i = 0
        self.t0 = time.perf_counter()
        while i < len(order) or self.pending():
            now = self.now()
            while i < len(order) and (order[i].arrival <= now or not realtime):
                if not realtime:
                    order[i].arrival = now
                self.submit(order[i])
                i += 1
            self.poll()
        torch.cuda.synchronize()
        return order

    # ------------------------------------------------------------ internals
    def _admit(self):
        while len(self.inflight) < self.max_inflight:
            # the queue whose oldest job arrived first
            best = None
            for key, q in self.queues.items():
                if q and (best is None or q[0].req.arrival < self.queues[best][0].req.arrival):
                    best = key
            if best is None:
                return
            dbname, st = best
            q = self.queues[best]
            jobs, Qsum = [], 0
            while q and Qsum + q[0].req.Q <= self.max_batch_queries:
                cand = jobs + [q[0]]
                M = sum(self._job_M(j) for j in cand)
                if self._footprint(dbname, st, Qsum + q[0].req.Q, M) + self.used > self.hbm_budget:
                    break
                jobs.append(q.popleft())
                Qsum += jobs[-1].req.Q
            if not jobs:
                if not self.inflight:
                    # nothing in flight and the head still does not fit: admit alone
                    jobs = [q.popleft()]
                else:
                    return
            self._launch(dbname, st, jobs)

    def _grow(self, pool: list, slot: int, nbytes: int, like: torch.Tensor) -> torch.Tensor:
        """The slot's buffer, reallocated (at least doubled, at least 64 MiB)
        when it is smaller than nbytes: a handful of allocations per pool
        over a run, so the caching allocator is not fragmented by buffers of
        every size."""
        buf = pool[slot]
        if buf is None or buf.numel() < nbytes:
            old = 0 if buf is None else buf.numel()
            pool[slot] = None
            buf = torch.empty(max(nbytes, 2 * old, 64 << 20), dtype=torch.uint8,
                              device=like.device)
            pool[slot] = buf
        return buf

    def _launch(self, dbname: str, st: str, jobs: List[_Job]):
        R = self.dbs[dbname]
        slot = self.busy.index(False)
        self.busy[slot] = True
        stream = self.streams[slot]
        self.launches += 1
        cts = [j.req.ct for j in jobs]
        qids = np.concatenate([j.req.qids for j in jobs]).astype(np.uint64)
        work = None
        if st == "points":
            sel = [s for j in jobs for s in j.req.selected]
            work = R.server.work_list(sel)
            desc_db, key = R.server.db, R.server.key_points
        elif st == "centres":
            desc_db, key = R.server.cdb, R.server.key_centers
        else:
            desc_db, key = R.db, R.key
        with torch.cuda.stream(stream):
            if len(cts) == 1:
                ct = cts[0]
            else:
                shape = (sum(c.shape[0] for c in cts),) + tuple(cts[0].shape[1:])
                nb = int(np.prod(shape)) * 8
                ct = self._grow(self.pool_ct, slot, nb, cts[0])[:nb].view(torch.uint64)
                ct = ct.view(shape)
                torch.cat(cts, dim=0, out=ct)
            qd = torch.as_tensor(qids).to(ct.device, non_blocking=False)
            need = nat.sanns_distances_workspace(R.ctx.handle, desc_db.desc, ct.shape[0],
                                                 ct.shape[0] * desc_db.n_chunks
                                                 if work is None else len(work), self.mode)
            ws = self._grow(self.pool_ws, slot, need, ct)
            outs = None
            if not self.keep_outputs:
                M = ct.shape[0] * desc_db.n_chunks if work is None else len(work)
                outs = (self._grow(self.pool_out, slot, M * 2 * R.ctx.L * R.ctx.N * 8, ct),
                        self._grow(self.pool_share, slot, M * R.ctx.N * 4, ct))
            D = stage.Distances(R.ctx, desc_db, ct.shape[0], work=work, mode=self.mode,
                                workspace=ws, out_buffers=outs)
            out, share = D.run(ct, key, qd, stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        nbytes = D.ws_bytes + out.numel() * 8 + share.numel() * 4
        self.used += nbytes
        self.peak_used = max(self.peak_used, self.used)
        self.inflight.append(_Launch(slot, jobs, dbname, st, nbytes, ev, stream, out, share,
                                     work, [ct, qd, D]))

    def _retire(self, lx: _Launch):
        self.used -= lx.bytes
        self.busy[lx.slot] = False
        C = self._n_chunks(lx.dbname, lx.stage)
        row = 0
        q0 = 0
        for j in lx.jobs:
            if lx.work is None:
                M = j.req.Q * C
                rows = slice(row, row + M)
            else:
                qs = np.arange(q0, q0 + j.req.Q)
                idx = np.nonzero(np.isin(lx.work[:, 0], qs))[0]
                rows = slice(int(idx[0]), int(idx[-1]) + 1)
                M = len(idx)
            wk = None
            if lx.work is not None:
                wk = lx.work[rows].copy()
                wk[:, 0] -= q0
            j.req.outputs[lx.stage] = (lx.out[rows], lx.share[rows], wk)
            row += M
            q0 += j.req.Q
            if lx.stage == "centres":
                j.req.phase = 1
                j.req.selected = self.client_select(j.req, self.dbs[j.req.db])
                if not self.keep_outputs:
                    j.req.outputs.pop("centres")
                self.queues[(j.req.db, "points")].append(_Job(j.req, "points"))
            else:
                j.req.done = self.now()
                if not self.keep_outputs:
                    j.req.outputs.clear()
                self.completed.append(j.req)


def latency_stats(reqs: Sequence[Request]) -> dict:
    lat = np.array([1e3 * (r.done - r.arrival) for r in reqs if r.done >= 0])
    return {"requests": int(len(lat)),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_ms": float(lat.mean()) if len(lat) else None}
