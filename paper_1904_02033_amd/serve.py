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

Query ids: the mask of a slot is drawn from (database key, query id, chunk),
so a (key, id) pair used for two different queries would hand the client two
masks that cancel.  The loop therefore assigns every query's id itself, from
a counter that belongs to the resident database (and lives as long as its
keys), and ignores ids a request may carry.

HBM admission counts everything the loop allocates on the device: the
per-slot pools (workspace, concatenated query ciphertexts, and output
buffers when outputs are released at completion) at their actual capacity,
plus the per-launch outputs and query-id vectors of launches in flight.

Latency is measured from a request's arrival to the moment its shares are
ready on the device.
"""
from __future__ import annotations

import collections
import dataclasses
import os
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
    key: bytes = b""                                    # empty: a fresh random key
    u: int = 64                                         # clusters per query
    next_qid: int = 0                                   # next unused query id under `key`

    def __post_init__(self):
        if self.server is None and not self.key:
            self.key = os.urandom(32)

    @property
    def clustered(self) -> bool:
        return self.server is not None

    def take_qids(self, Q: int) -> np.ndarray:
        """Q query ids never used before under this database's mask key(s)
        (a clustered index keeps the counter of its own two keys)."""
        if self.server is not None:
            return self.server.take_qids(Q)
        out = np.arange(self.next_qid, self.next_qid + Q, dtype=np.uint64)
        self.next_qid += Q
        return out


@dataclasses.dataclass
class Request:
    rid: int
    db: str
    ct: torch.Tensor            # [Q][d][2][L][N] query ciphertexts (device)
    k: int
    arrival: float = 0.0        # seconds since the loop started
    # filled in by the loop
    qids: Optional[np.ndarray] = None   # [Q] uint64 mask-stream ids assigned at submit
    error: Optional[str] = None         # set when a later stage could not be admitted
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


# Launches in flight at most.  Measured on the three-database trace: three
# and four trade p50 against p99 (see the design notes); six collapsed at 90%
# load (p50 0.6-0.9 s) while every slot kept its own pools of buffers.
MAX_INFLIGHT = 4


class Server:
    def __init__(self, dbs: Sequence[ResidentDB], hbm_budget: int, max_inflight: int = 3,
                 max_batch_queries: int = 64, mode: int = nat.SANNS_MODE_FUSED,
                 client_select: Optional[Callable] = None, keep_outputs: bool = True):
        """keep_outputs=False releases each request's output buffers when it
        completes (as a server does once the shares have been sent).
        max_inflight is capped at MAX_INFLIGHT."""
        if max_inflight < 1:
            raise ValueError("max_inflight must be at least 1")
        self.dbs = {d.name: d for d in dbs}
        self.hbm_budget = int(hbm_budget)
        self.max_inflight = min(max_inflight, MAX_INFLIGHT)
        max_inflight = self.max_inflight
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
    _POOLS = ("ws", "ct", "out", "share")

    def _pool(self, name: str) -> list:
        return {"ws": self.pool_ws, "ct": self.pool_ct, "out": self.pool_out,
                "share": self.pool_share}[name]

    def _pooled(self, name: str) -> bool:
        return name in ("ws", "ct") or not self.keep_outputs

    def _pool_total(self) -> int:
        return sum(b.numel() for n in self._POOLS for b in self._pool(n) if b is not None)

    def _live(self) -> int:
        return sum(lx.bytes for lx in self.inflight)

    def _desc(self, dbname: str, st: str) -> stage.Database:
        R = self.dbs[dbname]
        if st == "centres":
            return R.server.cdb
        if st == "points":
            return R.server.db
        return R.db

    def _sizes(self, dbname: str, st: str, Q: int, M: int, n_jobs: int) -> dict:
        """Device bytes of one launch of Q queries and M outputs: workspace,
        the concatenated query ciphertexts (launches of several jobs), output
        ciphertexts and shares, and the query-id vector (rounded up to the
        allocator's 512-byte granule)."""
        R = self.dbs[dbname]
        ctx = R.ctx
        db = self._desc(dbname, st)
        return {"ws": nat.sanns_distances_workspace(ctx.handle, db.desc, Q, M, self.mode),
                "ct": Q * db.d * 2 * ctx.L * ctx.N * 8 if n_jobs > 1 else 0,
                "out": M * 2 * ctx.L * ctx.N * 8,
                "share": M * ctx.N * 4,
                "qd": (Q * 8 + 511) // 512 * 512}

    def _footprint(self, dbname: str, st: str, Q: int, M: int) -> int:
        """Bytes one job needs when it is launched alone on empty pools."""
        return sum(self._sizes(dbname, st, Q, M, 1).values())

    def _plan(self, slot: int, sizes: dict):
        """Pool capacities slot `slot` gets for a launch of these sizes (the
        pools that must grow; geometric growth -- at least doubled, at least
        64 MiB -- only where it still fits the budget), the device bytes the
        loop then holds in total, and the launch's own unpooled bytes."""
        total = self._pool_total() + self._live()
        new_live = sizes["qd"]
        caps = {}
        for n in self._POOLS:
            if not self._pooled(n):
                new_live += sizes[n]
                continue
            buf = self._pool(n)[slot]
            cur = 0 if buf is None else buf.numel()
            if sizes[n] > cur:
                caps[n] = sizes[n]
                total += sizes[n] - cur
        total += new_live
        for n in caps:
            buf = self._pool(n)[slot]
            cur = 0 if buf is None else buf.numel()
            grown = max(caps[n], 2 * cur, 64 << 20)
            if total + grown - caps[n] <= self.hbm_budget:
                total += grown - caps[n]
                caps[n] = grown
        return caps, total, new_live

    def _n_chunks(self, dbname: str, st: str) -> int:
        return self._desc(dbname, st).n_chunks

    def _job_M(self, job: _Job) -> int:
        if job.stage == "points":
            return len(self.dbs[job.req.db].server.work_list(job.req.selected))
        return job.req.Q * self._n_chunks(job.req.db, job.stage)

    # ------------------------------------------------------------ interface
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: Request):
        """Queue a request.  Its query ids are assigned here, from the
        database's counter; a request that could not run even alone on an
        otherwise empty device budget raises AdmissionError."""
        R = self.dbs[req.db]
        st = "centres" if R.clustered else "scan"
        job = _Job(req, st)
        need = self._footprint(req.db, st, req.Q, self._job_M(job))
        if need > self.hbm_budget:
            raise AdmissionError(f"request {req.rid} needs {need} B > budget {self.hbm_budget} B")
        req.qids = R.take_qids(req.Q)
        self.queues[(req.db, st)].append(job)

    def pending(self) -> bool:
        return bool(self.inflight) or any(self.queues.values())

    def poll(self):
        """Retire finished launches, then admit queued work."""
        done = [lx for lx in self.inflight if lx.event.query()]
        self.inflight = [lx for lx in self.inflight if lx not in done]
        for lx in done:
            self._retire(lx)
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
            slot = self.busy.index(False)
            jobs, Qsum, M, plan = [], 0, 0, None
            while q and Qsum + q[0].req.Q <= self.max_batch_queries:
                Mc = M + self._job_M(q[0])
                sizes = self._sizes(dbname, st, Qsum + q[0].req.Q, Mc, len(jobs) + 1)
                cand = self._plan(slot, sizes)
                if cand[1] > self.hbm_budget:
                    break
                jobs.append(q.popleft())
                Qsum += jobs[-1].req.Q
                M, plan = Mc, cand
            if not jobs:
                if self.inflight:
                    return
                # nothing in flight and the head does not fit beside the idle
                # pools: release them; alone on empty pools it fits (checked
                # when it was queued)
                for n in self._POOLS:
                    pool = self._pool(n)
                    for i in range(len(pool)):
                        pool[i] = None
                jobs = [q.popleft()]
                plan = self._plan(slot, self._sizes(dbname, st, jobs[0].req.Q,
                                                    self._job_M(jobs[0]), 1))
            self._launch(dbname, st, jobs, slot, plan)

    def _grow(self, pool: list, slot: int, nbytes: int, caps: dict, name: str,
              like: torch.Tensor) -> torch.Tensor:
        """The slot's buffer of at least nbytes, reallocated at the capacity
        the admission planned when it is smaller."""
        buf = pool[slot]
        if buf is None or buf.numel() < nbytes:
            pool[slot] = None
            buf = torch.empty(caps[name], dtype=torch.uint8, device=like.device)
            pool[slot] = buf
        return buf

    def _launch(self, dbname: str, st: str, jobs: List[_Job], slot: int, plan):
        caps, _, new_live = plan
        R = self.dbs[dbname]
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
        Qn = sum(c.shape[0] for c in cts)
        M = Qn * desc_db.n_chunks if work is None else len(work)
        sizes = self._sizes(dbname, st, Qn, M, len(jobs))
        with torch.cuda.stream(stream):
            if len(cts) == 1:
                ct = cts[0]
            else:
                shape = (Qn,) + tuple(cts[0].shape[1:])
                nb = sizes["ct"]
                ct = self._grow(self.pool_ct, slot, nb, caps, "ct", cts[0])[:nb]
                ct = ct.view(torch.uint64).view(shape)
                torch.cat(cts, dim=0, out=ct)
            qd = torch.as_tensor(qids).to(ct.device, non_blocking=False)
            ws = self._grow(self.pool_ws, slot, sizes["ws"], caps, "ws", ct)
            outs = None
            if not self.keep_outputs:
                outs = (self._grow(self.pool_out, slot, sizes["out"], caps, "out", ct),
                        self._grow(self.pool_share, slot, sizes["share"], caps, "share", ct))
            D = stage.Distances(R.ctx, desc_db, Qn, work=work, mode=self.mode,
                                workspace=ws, out_buffers=outs)
            out, share = D.run(ct, key, qd, stream)
            ev = torch.cuda.Event()
            ev.record(stream)
        self.inflight.append(_Launch(slot, jobs, dbname, st, new_live, ev, stream, out, share,
                                     work, [ct, qd, D]))
        self.used = self._pool_total() + self._live()
        self.peak_used = max(self.peak_used, self.used)

    def _retire(self, lx: _Launch):
        self.busy[lx.slot] = False
        self.used = self._pool_total() + self._live()
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
                job = _Job(j.req, "points")
                need = self._footprint(j.req.db, "points", j.req.Q, self._job_M(job))
                if need > self.hbm_budget:
                    # its second stage can never run within the budget
                    j.req.error = f"points stage needs {need} B > budget {self.hbm_budget} B"
                    j.req.done = self.now()
                    self.completed.append(j.req)
                    continue
                self.queues[(j.req.db, "points")].append(job)
            else:
                j.req.done = self.now()
                if not self.keep_outputs:
                    j.req.outputs.clear()
                self.completed.append(j.req)


def latency_stats(reqs: Sequence[Request]) -> dict:
    lat = np.array([1e3 * (r.done - r.arrival) for r in reqs
                    if r.done >= 0 and r.error is None])
    return {"requests": int(len(lat)),
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else None,
            "mean_ms": float(lat.mean()) if len(lat) else None}
