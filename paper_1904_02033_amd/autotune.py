"""Schedule autotuner for sanns_distances.

For one call shape (ring, limbs, d, queries, chunks, all-pairs or work list)
it times every built schedule on the device with the caller's inputs:

  * SANNS_MODE_BATCHED (a hipGraph of the per-phase kernels) with each
    LDS-staged multiply-accumulate variant and, for contexts created with
    SANNS_FLAG_DIGIT_DB, the int8 matrix-core schedule (all-pairs), or each
    register tile (work lists),
  * SANNS_MODE_PERSISTENT (one work-queue launch) with each tile shape built
    for the ring degree,

checks that every schedule returns the same bytes as the first one (the
schedule never changes results), and applies the fastest to the context.
Results can be kept in a JSON cache keyed by device and call shape.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

from . import native as nat

# Multiply-accumulate schedules built into the library (ids as in sanns.h).
LDS_VARIANTS = list(range(1, 12)) + list(range(21, 28))   # all need N % 32 == 0
REGISTER_TILES = [(1, 1), (1, 2), (1, 4), (1, 8), (2, 2), (2, 4), (4, 2), (2, 3), (3, 2)]
MFMA_SCHEDULE = nat.SANNS_SCHEDULE_MFMA  # needs SANNS_FLAG_DIGIT_DB, d <= 128
MFMA_MAX_D = 128
# persistent tile shapes per log2 N, with the largest d each accumulates in one pass
PERSIST_SHAPES = {11: [(61, 252)], 12: [(51, 252), (52, 252)],
                  13: [(41, 252), (42, 252), (43, 252), (44, 252)], 14: [(71, 254)]}


@dataclasses.dataclass
class Schedule:
    mode: int
    variant: int = 0     # LDS variant (batched) or persistent shape
    qt: int = 0          # register tile for work lists (batched)
    ct: int = 0
    ms: float = float("nan")

    def label(self) -> str:
        if self.mode == nat.SANNS_MODE_PERSISTENT:
            return f"persistent/{self.variant}"
        if self.variant == MFMA_SCHEDULE:
            return "batched/mfma"
        if self.variant:
            return f"batched/lds{self.variant}"
        return f"batched/tile{self.qt}x{self.ct}"

    def apply(self, ctx) -> None:
        ctx.set_schedule(self.qt, self.ct, self.variant)


def candidates(ctx, d: int, regular: bool, Q: int) -> List[Schedule]:
    logN = ctx.N.bit_length() - 1
    out: List[Schedule] = []
    if regular and Q >= 2 and ctx.N % 32 == 0:
        out += [Schedule(nat.SANNS_MODE_BATCHED, v) for v in LDS_VARIANTS]
        if (ctx.params.flags & nat.SANNS_FLAG_DIGIT_DB) and d <= MFMA_MAX_D and ctx.N >= 64:
            out.append(Schedule(nat.SANNS_MODE_BATCHED, MFMA_SCHEDULE))
    else:
        out += [Schedule(nat.SANNS_MODE_BATCHED, 0, qt, ct) for qt, ct in REGISTER_TILES]
    out += [Schedule(nat.SANNS_MODE_PERSISTENT, s) for s, max_d in PERSIST_SHAPES.get(logN, [])
            if d <= max_d]
    return out


def cache_key(ctx, db, Q: int, work: Optional[np.ndarray]) -> str:
    import torch
    dev = torch.cuda.get_device_name(db.mem.device)
    M = Q * db.n_chunks if work is None else len(work)
    kind = "all" if work is None else "list"
    return f"{dev}|N={ctx.N}|L={ctx.L}|d={db.d}|Q={Q}|C={db.n_chunks}|M={M}|{kind}"


def _load(path: Optional[str]) -> Dict[str, dict]:
    if not path or not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def _save(path: Optional[str], table: Dict[str, dict]) -> None:
    if not path:
        return
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(ctx, db, ct_in, mask_key: bytes, query_ids, work: Optional[np.ndarray] = None,
         reps: int = 3, cands: Optional[Sequence[Schedule]] = None,
         cache_path: Optional[str] = None) -> Tuple[Schedule, List[Schedule]]:
    """Time the candidate schedules on (ct_in, query_ids), apply the fastest
    to ctx and return (best, every candidate with its time).  A cache hit
    returns the stored schedule without timing anything."""
    import torch
    from . import stage

    Q = int(ct_in.shape[0])
    key = cache_key(ctx, db, Q, work)
    table = _load(cache_path)
    if key in table:
        best = Schedule(**table[key])
        best.apply(ctx)
        return best, [best]
    if cands is None:
        cands = candidates(ctx, db.d, work is None, Q)
    ref = None
    timed: List[Schedule] = []
    for c in cands:
        c = dataclasses.replace(c)
        c.apply(ctx)
        D = stage.Distances(ctx, db, Q, work=work, mode=c.mode)
        D.run(ct_in, mask_key, query_ids)          # capture / warm-up
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            D.run(ct_in, mask_key, query_ids)
        e1.record()
        torch.cuda.synchronize()
        ctx.device_status()
        c.ms = e0.elapsed_time(e1) / reps
        got = (D.ct_out.view(torch.int64), D.share.view(torch.int32))
        if ref is None:
            ref = (got[0].clone(), got[1].clone())
        elif not (torch.equal(ref[0], got[0]) and torch.equal(ref[1], got[1])):
            raise RuntimeError(f"schedule {c.label()} changed the outputs")
        timed.append(c)
        del D
    best = min(timed, key=lambda s: s.ms)
    best.apply(ctx)
    if cache_path:
        table[key] = dataclasses.asdict(best)
        _save(cache_path, table)
    return best, timed
