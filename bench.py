"""Benchmark of the homomorphic distance stage on one MI355X.

Workload: linear scan of a resident 1,000,000 x 128 uint8 database (a
1,000-component Gaussian mixture, sigma 20, rounded and clipped; synthetic
stand-in for SIFT), BFV with N = 8192, three 54-bit primes, t = 16957441.
One step = one pass of the whole server hot path for a batch of 64 encrypted
queries: query NTTs, multiply-accumulate over every chunk of the resident
database, INTT, norm and mask, server shares out (the batched form, a cached
hipGraph).  Inputs are resident in HBM before the timed region.

Also measured and printed in the same JSON line: the plain form (one launch
per ciphertext operation) and the fused single-query form on the same
database, step and query latency percentiles, per-phase kernel times and the
roofline of the dominant kernel, and the CPU oracle timed on a one-chunk
sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import synthdata  # noqa: E402

METRIC = "encrypted distances/s at 1M×128 (batched vs plain); p50/p99 query latency"
UNIT = "encrypted distances/s"
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz 32-bit VALU lane-ops
VALU_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
HBM_PEAK_GBS = 8000.0


def device_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ["kernels.hip", "kernels.h", "modarith.h", "ntt.h"]:
        with open(os.path.join(ROOT, "paper_1904_02033_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the device source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "batched_1Mx128_q64_hbm_counters.md")
    try:
        text = open(path).read()
    except OSError:
        return None
    if device_source_hash() not in text:
        return None
    for line in text.splitlines():
        f = line.split()
        if len(f) == 3 and f[0] == "traffic_bytes_per_launch" and f[1] == kernel:
            return int(f[2])
    return None


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def pct(xs, p):
    return float(np.percentile(np.asarray(xs, dtype=np.float64), p))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--queries", type=int, default=64)
    ap.add_argument("--n", type=int, default=1_000_000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--plain-queries", type=int, default=1)
    ap.add_argument("--forms", default="batched,fused,plain",
                    help="comma list of forms to run besides the batched headline")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    args = ap.parse_args()
    forms = set(args.forms.split(","))
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the stage shards by database chunk; see the design notes)", flush=True)
        sys.exit(2)

    import torch
    from paper_1904_02033_amd import native as nat
    from paper_1904_02033_amd import stage

    if not os.path.exists(nat.LIB_PATH):
        from paper_1904_02033_amd import build as b
        b.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)

    w = synthdata.WORKLOADS[2]
    Q = args.queries
    t0 = time.time()
    pts = synthdata.gen_points(w, n=args.n)
    queries = synthdata.gen_queries(w, Q)
    n, d = pts.shape
    ctx = stage.Context(w.N, w.L, w.t_bits)
    N, L, t = ctx.N, ctx.L, ctx.t
    slot = stage.linear_slot_map(n, N, synthdata.gen_perm(n, synthdata.SEED_PERM + 2))
    db = stage.encode_db(ctx, pts, slot)
    C = db.n_chunks
    sk = torch.as_tensor(synthdata.gen_secret(N, synthdata.SEED_SK + 2)).to(dev)
    a = synthdata.gen_uniform_a(ctx.qs, N, Q * d, synthdata.SEED_ENC + 2)
    e = synthdata.gen_cbd_error(N, Q * d, synthdata.SEED_ENC + 2)
    ct = stage.encrypt_query(ctx, sk, torch.as_tensor(queries.astype(np.int32)).to(dev),
                             torch.as_tensor(a).to(dev), torch.as_tensor(e).to(dev))
    del a, e
    key = synthdata.gen_mask_key(synthdata.SEED_MASK + 2)
    qids = torch.as_tensor(np.arange(Q, dtype=np.uint64)).to(dev)
    torch.cuda.synchronize()
    log(f"setup {time.time() - t0:.1f}s: n={n} d={d} N={N} L={L} C={C} Q={Q}")

    # ---------------------------------------------------------------- batched
    B = stage.Distances(ctx, db, Q, mode=nat.SANNS_MODE_BATCHED)
    for _ in range(args.warmup):
        B.run(ct, key, qids)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for s in range(args.steps):
        evs[s][0].record()
        B.run(ct, key, qids)
        evs[s][1].record()
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    step_ms = [a_.elapsed_time(b_) for a_, b_ in evs]
    ms_per_step = 1e3 * t_total / args.steps
    dist_per_step = Q * n
    value = dist_per_step * args.steps / t_total
    ctx.device_status()
    log(f"batched: {ms_per_step:.3f} ms/step, {value / 1e9:.3f} G distances/s")

    # spot check: shares of query 0, chunk 0 reconstruct the true distances
    qn2 = np.array([int((queries[0].astype(np.int64) ** 2).sum()) % t], dtype=np.uint32)
    client = stage.decrypt_shares(ctx, sk, B.ct_out[:1].contiguous(),
                                  torch.as_tensor(qn2).to(dev))
    tot = (client.cpu().numpy()[0].astype(np.int64) +
           B.share[0].cpu().numpy().astype(np.int64)) % t
    ids = slot[:N]
    want = ((pts[ids].astype(np.int64) - queries[0].astype(np.int64)) ** 2).sum(axis=1)
    assert (tot == want).all(), "batched output does not decrypt to the true distances"

    # ------------------------------------------------- per-phase (roofline)
    nat.sanns_profile_enable(ctx.handle, True)
    for _ in range(3):
        B.run(ct, key, qids)
    phases, calls = nat.sanns_profile_read(ctx.handle)
    nat.sanns_profile_enable(ctx.handle, False)
    mulacc = Q * C * 2 * d * L * N
    mac_ms = phases["mac"]
    mac_ops = 3 * mulacc  # 32x32->64 multiply-adds: Karatsuba on 27-bit halves
    mac_tops = mac_ops / (mac_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "k_mac_lds", "achieved": round(mac_tops, 3),
                "peak": round(VALU_PEAK_TOPS, 3), "unit": "Tops/s (32-bit VALU lane-ops)",
                "frac": round(mac_tops / VALU_PEAK_TOPS, 4),
                "traffic": recorded_traffic("k_mac_lds"), "traffic_unit": "bytes/launch",
                "avg_ms": round(mac_ms, 4),
                "algorithmic": f"{mac_ops:.4g} ops = 3 x {mulacc:.4g} modular mul-acc"}
    log(f"phases (ms): {phases}")

    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        src.fill_(1)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    fused = plain = None
    plain_value = None
    # ----------------------------------------------------- fused, one query
    ct1 = ct[:1].contiguous()
    q1 = qids[:1].contiguous()
    F = stage.Distances(ctx, db, 1, mode=nat.SANNS_MODE_FUSED)
    if "fused" in forms or "plain" in forms:
        fused = run_fused(args, ctx, db, F, ct1, key, q1, n, d, L, C, N)

    # ----------------------------------------------------------- plain form
    if "plain" in forms:
        P = stage.Distances(ctx, db, 1, mode=nat.SANNS_MODE_PLAIN)
        P.run(ct1, key, q1)
        torch.cuda.synchronize()
        tp = time.perf_counter()
        for _ in range(args.plain_queries):
            P.run(ct1, key, q1)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp
        plain_value = n * args.plain_queries / tp
        assert (P.ct_out.cpu().numpy() == F.ct_out.cpu().numpy()).all() and \
            (P.share.cpu().numpy() == F.share.cpu().numpy()).all(), \
            "plain and fused forms disagree"
        plain = {"value": round(plain_value, 1), "unit": UNIT,
                 "ms_per_query": round(1e3 * tp / args.plain_queries, 2)}
        log(f"plain: {1e3 * tp / args.plain_queries:.1f} ms/query, "
            f"{plain_value / 1e6:.2f} M/s")

    # ------------------------------------------------------ CPU oracle leg
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, pts, slot, queries[0], N, L, t)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": f"batched linear scan: {n:,} x {d} uint8 Gaussian-mixture "
                               f"database, {Q} encrypted queries per step, BFV N={N}, "
                               f"L={L} x 54-bit primes, t={t}",
                   "n": n, "d": d, "queries_per_step": Q, "N": N, "L": L, "t": t,
                   "chunks": C, "form": "batched (hipGraph)", "parallelism": "single GPU"},
        "batched_vs_plain": round(value / plain_value, 1) if plain_value else None,
        "plain": plain,
        "fused_q1": fused,
        "latency": {"batched_step_p50_ms": round(pct(step_ms, 50), 3),
                    "batched_step_p99_ms": round(pct(step_ms, 99), 3),
                    "fused_query_p50_ms": fused["query_p50_ms"] if fused else None,
                    "fused_query_p99_ms": fused["query_p99_ms"] if fused else None},
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)
    ctx.close()


def run_fused(args, ctx, db, F, ct1, key, q1, n, d, L, C, N):
    import torch
    from paper_1904_02033_amd import native as nat
    for _ in range(3):
        F.run(ct1, key, q1)
    n_lat = max(10, args.steps)
    fev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n_lat)]
    torch.cuda.synchronize()
    tf = time.perf_counter()
    for s in range(n_lat):
        fev[s][0].record()
        F.run(ct1, key, q1)
        fev[s][1].record()
    torch.cuda.synchronize()
    tf = time.perf_counter() - tf
    q_ms = [a_.elapsed_time(b_) for a_, b_ in fev]
    fused_value = n * n_lat / tf
    nat.sanns_profile_enable(ctx.handle, True)
    for _ in range(3):
        F.run(ct1, key, q1)
    fph, _ = nat.sanns_profile_read(ctx.handle)
    nat.sanns_profile_enable(ctx.handle, False)
    db_bytes = L * C * d * N * 8
    q_bytes = d * 2 * L * N * 8
    out_bytes = C * 2 * L * N * 8
    mac1_bytes = db_bytes + q_bytes + out_bytes
    mac1_gbs = mac1_bytes / (fph["mac"] * 1e-3) / 1e9
    fused = {"value": round(fused_value, 1), "unit": UNIT,
             "query_p50_ms": round(pct(q_ms, 50), 3), "query_p99_ms": round(pct(q_ms, 99), 3),
             "phases_ms": {k: round(v, 4) for k, v in fph.items()},
             "roofline": {"bound": "hbm", "kernel": "k_mac", "achieved": round(mac1_gbs, 1),
                          "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": round(mac1_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                          "avg_ms": round(fph["mac"], 4),
                          "algorithmic": f"{mac1_bytes} B (resident DB + query NTT "
                                         "read + NTT-form outputs written)"}}
    log(f"fused Q=1: p50 {fused['query_p50_ms']} ms, {fused_value / 1e9:.3f} G/s, "
        f"mac {mac1_gbs:.0f} GB/s")
    return fused


def cpu_baseline(w, pts, slot, qv, N, L, t):
    """The oracle, as it stands, on one chunk (8192 slots) of this database
    for one query: its server stage (products, masks, norm plaintext) timed;
    its client encryption done first and not timed."""
    import oracle
    P = oracle.Params(N, oracle.rns_primes(N, L), t)
    assert P.t == t
    s = synthdata.gen_secret(N, 1)
    d = pts.shape[1]
    a = synthdata.gen_uniform_a(P.qs, N, d, 2)
    e = synthdata.gen_cbd_error(N, d, 2)
    ct = oracle.encrypt_constants(P, s, a, e, [int(x) for x in qv])
    g, nrm = oracle.chunk_plaintexts(pts, slot, N, 0)
    key = synthdata.gen_mask_key(3)
    t0 = time.perf_counter()
    oracle.server_chunk(P, ct, g, nrm, key, 0, 0)
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    log(f"cpu oracle: {dt:.2f}s for one chunk on {threads} threads")
    return {"value": round(N / dt, 1), "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"one chunk ({N} slots) of the {len(pts):,} x {d} database, one query: "
                      "schoolbook negacyclic products for 2 components x "
                      f"{L} limbs x {d} coordinates, masks and norm plaintext "
                      "(encryption not timed)",
            "seconds": round(dt, 2)}


if __name__ == "__main__":
    main()
