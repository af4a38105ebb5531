"""Benchmark of the homomorphic distance stage on one MI355X.

Workload: linear scan of a resident 1,000,000 x 128 uint8 database (a
1,000-component Gaussian mixture, sigma 20, rounded and clipped; synthetic
stand-in for SIFT), BFV with N = 8192, three 54-bit primes, t = 16957441.
One step = one pass of the whole server hot path for a batch of 64 encrypted
queries: query NTTs, multiply-accumulate over every chunk of the resident
database, INTT, norm and mask, server shares out.  The step runs in the
schedule the autotuner picks (a hipGraph of the per-phase kernels, with the
64-bit vector or the int8-digit matrix-core multiply-accumulate, or one
persistent work-queue launch, with their tile shapes), timed before the
measured region.  Inputs are resident in HBM before the timed region.

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
MFMA_I8_PEAK_TOPS = 5000.0  # dense int8 MFMA, MI355X
HBM_PEAK_GBS = 8000.0


def device_source_hash() -> str:
    """Hash of the device sources without their // comments and blank space,
    so that the recorded counters stay valid across comment edits and go
    stale on any change of code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in ["kernels.hip", "mfma.hip", "kernels.h", "modarith.h", "ntt.h", "chacha.h"]:
        with open(os.path.join(ROOT, "paper_1904_02033_amd", "csrc", f)) as fh:
            text = re.sub(r"//[^\n]*", "", fh.read())
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def recorded_traffic(kernel: str, summary: str = "batched_1Mx128_q64_hbm_counters.md"):
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter
    summary, or None when the device source changed since it was taken."""
    path = os.path.join(ROOT, "profiles", summary)
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


USE_DIGITS = True
T_POW2 = False  # --t-pow2: plain modulus 2^(t_bits - 1) instead of the prime


def digit_context(w):
    """Context of workload w whose databases also keep the int8 digit form
    that the matrix-core multiply-accumulate reads (SANNS_FLAG_DIGIT_DB),
    unless --no-digits."""
    from paper_1904_02033_amd import native as nat, stage
    params = nat.sanns_params_derive(w.N, w.L, w.t_bits)
    if USE_DIGITS:
        params.flags |= nat.SANNS_FLAG_DIGIT_DB
    if T_POW2:
        params.t = 1 << (w.t_bits - 1)
    return stage.Context(params=params)


def parse_schedule(text, nat, autotune):
    """'' (library default), 'mfma', 'lds<id>' or 'persistent/<id>'."""
    if not text:
        return autotune.Schedule(nat.SANNS_MODE_BATCHED)
    if text == "mfma":
        return autotune.Schedule(nat.SANNS_MODE_BATCHED, autotune.MFMA_SCHEDULE)
    if text.startswith("lds"):
        return autotune.Schedule(nat.SANNS_MODE_BATCHED, int(text[3:]))
    if text.startswith("persistent/"):
        return autotune.Schedule(nat.SANNS_MODE_PERSISTENT, int(text.split("/")[1]))
    raise SystemExit(f"unknown schedule {text!r}")


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
    ap.add_argument("--forms", default="batched,private,fused,plain",
                    help="comma list of forms to run besides the batched headline")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="also run one device copy of this many MiB (counter calibration)")
    ap.add_argument("--workload", default="batched-1Mx128",
                    choices=["batched-1Mx128", "batched-1Mx96", "linear-10Kx128",
                             "clustered-10M", "serving", "balance-1Mx96"])
    ap.add_argument("--serving-requests", type=int, default=200)
    ap.add_argument("--serving-budget-gib", type=float, default=0.0,
                    help="HBM budget of the serving loop's request buffers "
                         "(0: 75%% of the device memory free once the databases are resident)")
    ap.add_argument("--balance-m", type=int, default=22,
                    help="balance-1Mx96: largest cluster size m (the paper's Deep1B-1M value)")
    ap.add_argument("--balance-alpha", type=float, default=0.5)
    ap.add_argument("--balance-iters", type=int, default=8)
    ap.add_argument("--serving-rate", type=float, default=0.0,
                    help="also serve one Poisson trace at this absolute rate (req/s)")
    ap.add_argument("--no-tune", action="store_true",
                    help="skip the autotuner and run the library's default batched schedule "
                         "(used for profiler runs)")
    ap.add_argument("--no-digits", action="store_true",
                    help="create contexts without SANNS_FLAG_DIGIT_DB (vector schedules only)")
    ap.add_argument("--t-pow2", action="store_true",
                    help="plain modulus t = 2^(t_bits - 1), a power of two as in the paper's "
                         "parameters, instead of the prime t = 1 mod 2N")
    ap.add_argument("--schedule", default="",
                    help="with --no-tune: run this schedule instead of the default "
                         "(mfma, lds<id>, persistent/<id>)")
    args = ap.parse_args()
    global USE_DIGITS, T_POW2
    USE_DIGITS = not args.no_digits
    T_POW2 = args.t_pow2
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the stage shards by database chunk; see the design notes)", flush=True)
        sys.exit(2)
    import torch
    from paper_1904_02033_amd import native as nat
    if not os.path.exists(nat.LIB_PATH):
        from paper_1904_02033_amd import build as b
        b.build()
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.workload == "clustered-10M":
        line = run_clustered(args)
    elif args.workload == "serving":
        line = run_serving(args)
    elif args.workload == "balance-1Mx96":
        line = run_balance(args)
    else:
        cid = {"batched-1Mx128": 2, "batched-1Mx96": 3, "linear-10Kx128": 1}[args.workload]
        line = run_linear(args, synthdata.WORKLOADS[cid])
    print(json.dumps(line), flush=True)


def run_linear(args, w):
    forms = set(args.forms.split(","))
    import torch
    from paper_1904_02033_amd import native as nat
    from paper_1904_02033_amd import stage

    dev = torch.device("cuda", 0)
    Q = args.queries if w.cid != 1 else 1
    t0 = time.time()
    pts = synthdata.gen_points(w, n=args.n if w.cid != 1 else w.n)
    queries = synthdata.gen_queries(w, Q)
    n, d = pts.shape
    ctx = digit_context(w)
    N, L, t = ctx.N, ctx.L, ctx.t
    slot = synthdata.gen_slot_map(n, N, synthdata.SEED_PERM + w.cid)
    db = stage.encode_db(ctx, pts, slot)
    C = db.n_chunks
    sk = torch.as_tensor(synthdata.gen_secret(N, synthdata.SEED_SK + w.cid)).to(dev)
    a = synthdata.gen_uniform_a(ctx.qs, N, Q * d, synthdata.SEED_ENC + w.cid)
    e = synthdata.gen_cbd_error(N, Q * d, synthdata.SEED_ENC + w.cid)
    ct = stage.encrypt_query(ctx, sk, torch.as_tensor(queries.astype(np.int32)).to(dev),
                             torch.as_tensor(a).to(dev), torch.as_tensor(e).to(dev))
    del a, e
    key = synthdata.gen_mask_key(synthdata.SEED_MASK + w.cid)
    qids = torch.as_tensor(np.arange(Q, dtype=np.uint64)).to(dev)
    torch.cuda.synchronize()
    log(f"setup {time.time() - t0:.1f}s: n={n} d={d} N={N} L={L} C={C} Q={Q}")

    # ------------------------------------------------ schedule (autotuned)
    from paper_1904_02033_amd import autotune
    tt = time.time()
    if args.no_tune:
        best = parse_schedule(args.schedule, nat, autotune)
        best.apply(ctx)
        best.ms = float("nan")
        timed = [best]
    else:
        best, timed = autotune.tune(ctx, db, ct, key, qids, reps=3)
    log(f"autotune {time.time() - tt:.1f}s: best {best.label()} {best.ms:.3f} ms; " +
        ", ".join(f"{c.label()} {c.ms:.2f}" for c in sorted(timed, key=lambda c: c.ms)[:6]))

    # ---------------------------------------------------------------- batched
    B = stage.Distances(ctx, db, Q, mode=best.mode)
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
    real = ids >= 0
    want = ((pts[ids[real]].astype(np.int64) - queries[0].astype(np.int64)) ** 2).sum(axis=1)
    assert (tot[real] == want).all(), "batched output does not decrypt to the true distances"

    # ------------------------------------------------- per-phase (roofline)
    # Phases are timed on the fastest per-phase-kernel schedule (the
    # persistent form is one kernel and has no phase boundaries).
    batched = [c for c in timed if c.mode == nat.SANNS_MODE_BATCHED]
    pbest = min(batched, key=lambda c: c.ms) if batched else best
    pbest.apply(ctx)
    PB = stage.Distances(ctx, db, Q, mode=nat.SANNS_MODE_BATCHED)
    nat.sanns_profile_enable(ctx.handle, True)
    for _ in range(3):
        PB.run(ct, key, qids)
    phases, calls = nat.sanns_profile_read(ctx.handle)
    nat.sanns_profile_enable(ctx.handle, False)
    del PB
    best.apply(ctx)
    mulacc = Q * C * 2 * d * L * N
    mac_ms = phases["mac"]
    # the library's default all-pairs schedule: matrix cores on a digit database
    default = autotune.MFMA_SCHEDULE if (d <= autotune.MFMA_MAX_D and Q >= 2) else 22
    variant = pbest.variant or default
    traffic = None
    if variant == autotune.MFMA_SCHEDULE and Q >= 2:
        # int8 matrix cores: 49 digit-pair products per modular multiply-add
        mac_kernel = "k_mac_mfma"
        mac_ops = 2 * 49 * mulacc
        mac_tops = mac_ops / (mac_ms * 1e-3) / 1e12
        roofline = {"bound": "mfma", "kernel": mac_kernel,
                    "achieved": round(mac_tops, 3), "peak": MFMA_I8_PEAK_TOPS,
                    "unit": "TOPS (int8 MFMA, dense)",
                    "frac": round(mac_tops / MFMA_I8_PEAK_TOPS, 4),
                    "algorithmic": f"{mac_ops:.4g} int8 ops = 2 x 49 x {mulacc:.4g} "
                                   "digit-pair multiply-adds"}
    else:
        mac_ops = 3 * mulacc  # 32x32->64 multiply-adds: Karatsuba on 27-bit halves
        mac_kernel = "k_mac_dl" if variant >= 21 else "k_mac_lds"
        if Q < 2:
            mac_kernel = "k_mac"
        if best.mode == nat.SANNS_MODE_PERSISTENT:
            mac_ms, mac_kernel = pct(step_ms, 50), "k_persistent (whole step)"
        mac_tops = mac_ops / (mac_ms * 1e-3) / 1e12
        roofline = {"bound": "alu", "kernel": mac_kernel,
                    "achieved": round(mac_tops, 3),
                    "peak": round(VALU_PEAK_TOPS, 3), "unit": "Tops/s (32-bit VALU lane-ops)",
                    "frac": round(mac_tops / VALU_PEAK_TOPS, 4),
                    "algorithmic": f"{mac_ops:.4g} ops = 3 x {mulacc:.4g} modular mul-acc"}
    if w.cid == 2 and Q == 64:
        traffic = recorded_traffic(mac_kernel.split()[0])
    roofline.update({"traffic": traffic, "traffic_unit": "bytes/launch",
                     "avg_ms": round(mac_ms, 4),
                     # the same launch in the method's own units
                     "modular_mul_acc_per_s": round(mulacc / (mac_ms * 1e-3), 1),
                     "distances_per_s_in_kernel": round(Q * n / (mac_ms * 1e-3), 1)})
    if traffic:
        roofline["hbm_gbs"] = round(traffic / (mac_ms * 1e-3) / 1e9, 1)
    log(f"phases (ms): {phases}")

    # ------------------------------------- circuit-private form (same batch)
    private = None
    if "private" in forms and Q >= 1:
        private = run_private(args, ctx, db, pbest, ct, key, qids, sk, queries, slot, pts,
                              value, ms_per_step)
        best.apply(ctx)

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

    kind = "uint8" if pts.dtype == np.uint8 else "int8"
    headline = w.cid == 2 and Q == 64 and n == 1_000_000
    line = {
        "metric": METRIC if headline else
        f"encrypted distances/s at {n:,}x{d} {kind}, {Q} queries per step",
        "value": round(value, 1), "unit": UNIT, "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u64" if not best.label().endswith("mfma") else "u64 (int8 digit MFMA)",
        "data": "synthetic",
        "config": {"workload": f"batched linear scan: {n:,} x {d} {kind} ({w.gen}) "
                               f"database, {Q} encrypted queries per step, BFV N={N}, "
                               f"L={L} x 54-bit primes, t={t}",
                   "n": n, "d": d, "queries_per_step": Q, "N": N, "L": L, "t": t,
                   "chunks": C, "parallelism": "single GPU",
                   "form": f"{best.label()} (hipGraph; autotuned over {len(timed)} schedules)",
                   "schedules_ms": {c.label(): round(c.ms, 3)
                                    for c in sorted(timed, key=lambda c: c.ms)}},
        "batched_vs_plain": round(value / plain_value, 1) if plain_value else None,
        "plain": plain,
        "fused_q1": fused,
        "latency": {"batched_step_p50_ms": round(pct(step_ms, 50), 3),
                    "batched_step_p99_ms": round(pct(step_ms, 99), 3),
                    "fused_query_p50_ms": fused["query_p50_ms"] if fused else None,
                    "fused_query_p99_ms": fused["query_p99_ms"] if fused else None},
        "phases_ms": {k: round(v, 4) for k, v in phases.items()},
        "ntts_per_s": {"forward": round(Q * d * 2 * L / (phases["query_ntt"] * 1e-3), 1),
                       "inverse": round(Q * C * 2 * L / (phases["intt_mask"] * 1e-3), 1),
                       "N": N},
        "roofline": roofline if Q > 1 or not fused else fused["roofline"],
        "cpu_baseline": cpu,
        "private_form": private,
    }
    ctx.close()
    return line


def run_private(args, ctx, db, sched, ct, key, qids, sk, queries, slot, pts, value,
                ms_per_step):
    """The same batch in the circuit-private form (re-randomisation under the
    client's public key plus noise flooding): step time, distances/s and the
    cost over the plain batched step; every query shares one client's key."""
    import torch
    from paper_1904_02033_amd import native as nat, stage
    Q, N, t = ct.shape[0], ctx.N, ctx.t
    sched.apply(ctx)
    pk = stage.public_key(ctx, sk, 4321)
    pks = pk[None].expand(Q, *pk.shape).contiguous()
    D = stage.Distances(ctx, db, Q, mode=nat.SANNS_MODE_BATCHED, private=True)
    for _ in range(args.warmup):
        D.run(ct, key, qids, pk=pks)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        D.run(ct, key, qids, pk=pks)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ctx.device_status()
    # the shares of query 0, chunk 0 still reconstruct the true distances
    qn2 = np.array([int((queries[0].astype(np.int64) ** 2).sum()) % t], dtype=np.uint32)
    client = stage.decrypt_shares(ctx, sk, D.ct_out[:1].contiguous(),
                                  torch.as_tensor(qn2).to(ct.device))
    tot = (client.cpu().numpy()[0].astype(np.int64) +
           D.share[0].cpu().numpy().astype(np.int64)) % t
    ids = slot[:N]
    real = ids >= 0
    want = ((pts[ids[real]].astype(np.int64) - queries[0].astype(np.int64)) ** 2).sum(axis=1)
    assert (tot[real] == want).all(), "private form does not decrypt to the distances"
    nat.sanns_profile_enable(ctx.handle, True)
    for _ in range(3):
        D.run(ct, key, qids, pk=pks)
    ph, _ = nat.sanns_profile_read(ctx.handle)
    nat.sanns_profile_enable(ctx.handle, False)
    v = Q * len(pts) / dt
    b = nat.sanns_flood_bits(ctx.handle)
    log(f"private form: {1e3 * dt:.3f} ms/step, {v / 1e9:.3f} G distances/s "
        f"(flood 2^{b}); phases {ph}")
    return {"value": round(v, 1), "unit": UNIT, "ms_per_step": round(1e3 * dt, 4),
            "cost_vs_batched": round(1e3 * dt / ms_per_step, 3), "flood_bits": b,
            "schedule": sched.label(),
            "phases_ms": {k: round(x, 4) for k, x in ph.items()}}


def run_balance(args):
    """Balanced clustering (Section 3.3) of a 1M x 96 int8 database shaped
    like Deep1B-1M (the paper's setting for it: clusters of at most m = 22
    points): the k-means rounds on the GPU, the search over k on the host."""
    import torch
    from paper_1904_02033_amd import balance
    w = synthdata.WORKLOADS[3]
    n = args.n
    pts = synthdata.gen_points(w, n=n)
    d = pts.shape[1]
    m, alpha, iters = args.balance_m, args.balance_alpha, args.balance_iters
    perm = lambda level, k: synthdata.gen_perm(k, synthdata.SEED_PERM + 30 + level)
    dev = torch.device("cuda", 0)
    # one k-means round at the first level's lower-bound k, timed on its own
    k0 = max(1, int(np.ceil((1 - alpha) * n / m)))
    from paper_1904_02033_amd import native as nat
    km = balance.KMeans(torch.as_tensor(pts).to(dev))
    C, a, _ = km.run(perm(0, n)[:k0], 1)
    ws = km._ws(k0)
    s = torch.cuda.current_stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for rep in range(2):  # the first launch warms up
        ev[0].record()
        nat.sanns_kmeans_assign(km.X.data_ptr(), n, d, C.data_ptr(), k0, 0, a.data_ptr(), 0,
                                ws.data_ptr(), ws.numel(), s.cuda_stream)
        ev[1].record()
        torch.cuda.synchronize()
    round_ms = ev[0].elapsed_time(ev[1])
    pairs = n * k0
    dot4 = 2 * ((d + 3) // 4)
    lane_ops = pairs * dot4 / (round_ms * 1e-3) / 1e12
    log(f"k-means assignment: n={n} k={k0} d={d}: {round_ms:.2f} ms, "
        f"{pairs / (round_ms * 1e-3) / 1e9:.1f} G point-centre pairs/s")
    t0 = time.perf_counter()
    res = balance.balanced_clustering(pts, m, alpha, iters, perm)
    dt = time.perf_counter() - t0
    groups = [{"k_searched": g.k_searched, "clusters": int(len(g.centers)),
               "points": int(len(g.point_ids)),
               "max_cluster": int(np.bincount(g.cluster).max())} for g in res.groups]
    # plain k-means with the same total number of clusters, for the
    # max-cluster-size reduction the balancing buys
    ktot = sum(gr["clusters"] for gr in groups)
    Cp, ap, _ = km.run(perm(0, n)[:ktot], iters)
    plain_max = int(np.bincount(ap.cpu().numpy()).max())
    bal_max = max(gr["max_cluster"] for gr in groups)
    log(f"balanced clustering: {dt:.1f} s, {len(groups)} groups, {res.kmeans_runs} k-means "
        f"runs, max cluster {bal_max} (plain k-means with {ktot} centres: {plain_max})")
    return {
        "metric": "balanced clustering (Section 3.3): k-means point-centre pairs/s and "
                  "total time",
        "value": round(pairs / (round_ms * 1e-3), 1), "unit": "point-centre pairs/s",
        "n_gpus": 1, "steps": 1, "warmup": 1, "ms_per_step": round(round_ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int8 dot4 / int64", "data": "synthetic",
        "config": {"workload": f"balanced clustering of {n:,} x {d} int8 (unit-norm x 127), "
                               f"m={m}, alpha={alpha}, {iters} k-means rounds at most",
                   "n": n, "d": d, "m": m, "alpha": alpha, "iters": iters},
        "kmeans_assign": {"k": k0, "ms": round(round_ms, 3),
                         "roofline": {"bound": "alu", "kernel": "k_km_assign",
                                      "achieved": round(lane_ops, 3),
                                      "peak": round(VALU_PEAK_TOPS, 3),
                                      "unit": "T lane-ops/s (v_dot4_i32_i8)",
                                      "frac": round(lane_ops / VALU_PEAK_TOPS, 4),
                                      "algorithmic": f"{dot4} dot4 per point-centre pair"}},
        "balanced": {"seconds": round(dt, 2), "groups": groups, "kmeans_runs": res.kmeans_runs,
                     "kmeans_rounds": res.kmeans_rounds, "max_cluster": bal_max,
                     "plain_kmeans_max_cluster": plain_max, "total_clusters": ktot},
    }


def encrypt_pool(ctx, queries, seed, dev):
    """Client-side encryption of a pool of queries (not timed)."""
    import torch
    from paper_1904_02033_amd import stage
    Q, d = queries.shape
    sk = torch.as_tensor(synthdata.gen_secret(ctx.N, seed)).to(dev)
    a = synthdata.gen_uniform_a(ctx.qs, ctx.N, Q * d, seed + 1)
    e = synthdata.gen_cbd_error(ctx.N, Q * d, seed + 1)
    ct = stage.encrypt_query(ctx, sk, torch.as_tensor(queries.astype(np.int32)).to(dev),
                             torch.as_tensor(a).to(dev), torch.as_tensor(e).to(dev))
    torch.cuda.synchronize()
    return sk, ct


def clustered_world(dev, n_clusters=16384, total=9_900_000, stash=100_000):
    from paper_1904_02033_amd import clustered, stage
    w = synthdata.WORKLOADS[4]
    t0 = time.time()
    cdb = synthdata.gen_clustered(n_clusters=n_clusters, total_clustered=total, stash=stash,
                                  d=w.d, seed=synthdata.SEED_DATA + 4)
    ctx = digit_context(w)
    srv = clustered.ClusteredServer(
        ctx, cdb.points, cdb.cluster_sizes, cdb.centers, cdb.stash_size,
        synthdata.gen_perm(n_clusters, synthdata.SEED_PERM + 4),
        synthdata.gen_perm(stash, synthdata.SEED_PERM + 40),
        synthdata.gen_mask_key(synthdata.SEED_MASK + 4),
        synthdata.gen_mask_key(synthdata.SEED_MASK + 40))
    log(f"clustered setup {time.time() - t0:.1f}s: {len(cdb.points):,} points, "
        f"{srv.db.n_chunks} chunks, {srv.cdb.n_chunks} centre chunks")
    return w, cdb, ctx, srv


def client_select_fn(srv, sk, queries_of, u):
    """Client step between the two phases: decrypt the centre shares and
    pick the u closest clusters per query (cleartext stand-in)."""
    import torch
    from paper_1904_02033_amd import clustered, stage

    side = torch.cuda.Stream()

    def select(req_or_pair, R=None):
        with torch.cuda.stream(side):
            return _select(req_or_pair, R)

    def _select(req_or_pair, R=None):
        if R is not None:  # serving loop: a request
            out, share, _ = req_or_pair.outputs["centres"]
            qs = queries_of(req_or_pair)
        else:
            out, share, qs = req_or_pair
        ctx = srv.ctx
        C = srv.cdb.n_chunks
        qn2 = ((qs.astype(np.int64) ** 2).sum(axis=1) % ctx.t).astype(np.uint32)
        cl = stage.decrypt_shares(ctx, sk, out.contiguous(),
                                  torch.as_tensor(np.repeat(qn2, C)).to(out.device))
        cl, sh = cl.cpu().numpy(), share.cpu().numpy()
        sel = []
        for q in range(len(qs)):
            dist = ((cl[q * C:(q + 1) * C].astype(np.int64) + sh[q * C:(q + 1) * C])
                    % ctx.t).reshape(-1)
            sel.append(clustered.select_clusters(dist, srv.center_slot, u))
        return sel
    return select


def run_clustered(args):
    """Clustered sublinear form: 10M x 96 int8 in 16,384 Zipf clusters plus
    a 1% stash; 32 queries per launch, 64 clusters per query."""
    import torch
    from paper_1904_02033_amd import clustered, native as nat, stage
    dev = torch.device("cuda", 0)
    w, cdb, ctx, srv = clustered_world(dev)
    Q, u = w.Q, 64
    queries = synthdata.gen_queries(w, Q)
    sk, ct = encrypt_pool(ctx, queries, synthdata.SEED_SK + 4, dev)
    qids = torch.as_tensor(np.arange(Q, dtype=np.uint64)).to(dev)
    select = client_select_fn(srv, sk, None, u)
    # phase 1 once to fix the selection (client side between phases)
    cout, cshare = srv.center_distances(ct, qids)
    selected = select((cout, cshare, queries))
    work = srv.work_list(selected)
    # phase 2's per-query chunk lists get their own tuned schedule (register
    # tile or persistent shape); phase 1 keeps the default all-pairs one
    from paper_1904_02033_amd import autotune
    best2, timed2 = autotune.tune(ctx, srv.db, ct, srv.key_points, qids, work=work, reps=2)
    log(f"phase-2 autotune: {best2.label()} " +
        ", ".join(f"{c.label()} {c.ms:.2f}" for c in sorted(timed2, key=lambda c: c.ms)))
    D1 = stage.Distances(ctx, srv.cdb, Q, mode=nat.SANNS_MODE_BATCHED)
    D2 = stage.Distances(ctx, srv.db, Q, work=work, mode=best2.mode)
    for _ in range(args.warmup):
        D1.run(ct, srv.key_centers, qids)
        D2.run(ct, srv.key_points, qids)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    p1, p2 = [], []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e[0].record()
        D1.run(ct, srv.key_centers, qids)
        e[1].record()
        D2.run(ct, srv.key_points, qids)
        e[2].record()
        torch.cuda.synchronize()
        p1.append(e[0].elapsed_time(e[1]))
        p2.append(e[1].elapsed_time(e[2]))
    dt = (time.perf_counter() - t0) / args.steps
    srv.ctx.device_status()
    req_pairs = srv.requested_pairs(selected) + Q * srv.n_clusters
    slots = len(work) * ctx.N + Q * srv.cdb.n_chunks * ctx.N
    # spot check: one query's selected-cluster distances reconstruct exactly
    q = 0
    rows = np.nonzero(work[:, 0] == q)[0][:2]
    qn2 = np.array([int((queries[q].astype(np.int64) ** 2).sum()) % ctx.t] * len(rows),
                   dtype=np.uint32)
    cl = stage.decrypt_shares(ctx, sk, D2.ct_out[rows[0]:rows[-1] + 1].contiguous(),
                              torch.as_tensor(qn2).to(dev)).cpu().numpy()
    sh = D2.share[rows[0]:rows[-1] + 1].cpu().numpy()
    for i, m in enumerate(rows):
        ids = srv.layout.slot_point[work[m, 1] * ctx.N:(work[m, 1] + 1) * ctx.N]
        real = ids >= 0
        want = ((cdb.points[ids[real]].astype(np.int64) - queries[q]) ** 2).sum(axis=1)
        assert (((cl[i].astype(np.int64) + sh[i]) % ctx.t)[real] == want).all()
    lens = np.bincount(work[:, 0], minlength=Q)

    # phase 2 on per-query gathered chunks (clusters) plus the resident stash
    gsrv = clustered.ClusteredServer(
        ctx, cdb.points, cdb.cluster_sizes, cdb.centers, cdb.stash_size,
        synthdata.gen_perm(srv.n_clusters, synthdata.SEED_PERM + 4),
        synthdata.gen_perm(cdb.stash_size, synthdata.SEED_PERM + 40),
        synthdata.gen_mask_key(synthdata.SEED_MASK + 41), srv.key_centers, gathered=True)
    for _ in range(args.warmup):
        gsrv.point_distances_gathered(ct, qids, selected)
    torch.cuda.synchronize()
    pg = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        e[0].record()
        D1.run(ct, srv.key_centers, qids)
        e[1].record()
        (co, cs, gslot, grq), (so, ss) = gsrv.point_distances_gathered(ct, qids, selected)
        e[2].record()
        torch.cuda.synchronize()
        pg.append(e[1].elapsed_time(e[2]))
    dtg = (time.perf_counter() - t0) / args.steps
    gsrv.ctx.device_status()
    slots_g = (len(grq) + Q * gsrv.sdb.n_chunks) * ctx.N + Q * srv.cdb.n_chunks * ctx.N
    # spot check: query 0's first gathered chunk reconstructs exactly
    m0 = int(np.nonzero(grq == 0)[0][0])
    cl = stage.decrypt_shares(ctx, sk, co[m0:m0 + 1].contiguous(),
                              torch.as_tensor(qn2[:1]).to(dev)).cpu().numpy()[0]
    ids = gslot[m0 * ctx.N:(m0 + 1) * ctx.N].cpu().numpy()
    real = ids >= 0
    want = ((cdb.points[ids[real]].astype(np.int64) - queries[0]) ** 2).sum(axis=1)
    assert (((cl.astype(np.int64) + cs[m0].cpu().numpy()) % ctx.t)[real] == want).all()
    log(f"clustered: resident phase 2 {pct(p2, 50):.3f} ms ({slots} slots), gathered "
        f"phase 2 {pct(pg, 50):.3f} ms ({slots_g} slots)")
    gathered_better = dtg < dt
    return {
        "metric": "encrypted distances/s, clustered sublinear form (requested pairs)",
        "value": round(req_pairs / min(dt, dtg), 1), "unit": UNIT,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * min(dt, dtg), 3), "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": f"clustered: {len(cdb.points):,} x {w.d} int8, "
                               f"{srv.n_clusters} Zipf clusters + {cdb.stash_size:,} stash, "
                               f"{Q} queries x {u} clusters, N={ctx.N}, L={ctx.L}, t={ctx.t}",
                   "phase2": "gathered per-query chunks + resident stash" if gathered_better
                             else "resident cluster-packed chunks",
                   "chunks": srv.db.n_chunks, "centre_chunks": srv.cdb.n_chunks,
                   "phase2_form": best2.label(),
                   "phase2_schedules_ms": {c.label(): round(c.ms, 3)
                                           for c in sorted(timed2, key=lambda c: c.ms)}},
        "requested_pairs_per_step": int(req_pairs),
        "slots_processed_per_step": int(slots),
        "phase1_ms_p50": round(pct(p1, 50), 3), "phase2_ms_p50": round(pct(p2, 50), 3),
        "chunks_per_query": {"min": int(lens.min()), "median": float(np.median(lens)),
                             "max": int(lens.max())},
        "slot_throughput": round(slots / dt, 1),
        "resident": {"ms_per_step": round(1e3 * dt, 3), "value": round(req_pairs / dt, 1),
                     "phase2_ms_p50": round(pct(p2, 50), 3), "slots_processed": int(slots),
                     "requested_over_processed": round(req_pairs / slots, 4)},
        "gathered": {"ms_per_step": round(1e3 * dtg, 3), "value": round(req_pairs / dtg, 1),
                     "phase2_ms_p50": round(pct(pg, 50), 3), "slots_processed": int(slots_g),
                     "gathered_chunks": int(len(grq)), "stash_chunks": int(gsrv.sdb.n_chunks),
                     "requested_over_processed": round(req_pairs / slots_g, 4)},
    }


def run_serving(args):
    """Serving: Poisson arrivals against three resident databases; p50/p99
    arrival-to-shares latency and distances/s, against the per-query path."""
    import torch
    from paper_1904_02033_amd import native as nat, serve, stage
    dev = torch.device("cuda", 0)
    wA, wB = synthdata.WORKLOADS[2], synthdata.WORKLOADS[3]
    ctxA = digit_context(wA)
    ptsA = synthdata.gen_points(wA, n=100_000, seed=synthdata.SEED_DATA + 5)
    dbA = stage.encode_db(ctxA, ptsA, stage.linear_slot_map(
        len(ptsA), ctxA.N, synthdata.gen_perm(len(ptsA), synthdata.SEED_PERM + 5)))
    w4, cdb, ctxB, srv = clustered_world(dev)
    ptsB = synthdata.gen_points(wB)
    dbB = stage.encode_db(ctxB, ptsB, stage.linear_slot_map(
        len(ptsB), ctxB.N, synthdata.gen_perm(len(ptsB), synthdata.SEED_PERM + 3)))
    pool = 64
    qA = synthdata.gen_queries(wA, pool)
    qB = synthdata.gen_queries(wB, pool)
    skA, ctA = encrypt_pool(ctxA, qA, synthdata.SEED_SK + 5, dev)
    skB, ctB = encrypt_pool(ctxB, qB, synthdata.SEED_SK + 50, dev)
    dbs = [serve.ResidentDB("A", ctxA, db=dbA, key=synthdata.gen_mask_key(5001)),
           serve.ResidentDB("B", ctxB, db=dbB, key=synthdata.gen_mask_key(5002)),
           serve.ResidentDB("C", ctxB, server=srv, u=64)]
    n_of = {"A": len(ptsA), "B": len(ptsB)}
    select = client_select_fn(srv, skB, lambda r: qB[r.pool_rows], 64)
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if args.serving_budget_gib > 0:
        budget = int(args.serving_budget_gib * (1 << 30))
    else:
        budget = int(0.75 * torch.cuda.mem_get_info(dev)[0])
    log(f"serving budget {budget / (1 << 30):.1f} GiB for request buffers")

    def make_requests(rate, count, seed, per_query=False):
        """Requests of the arrival trace; with per_query every request is
        split into single-query requests that share its arrival time."""
        arr = synthdata.gen_arrivals(count, rate, n_dbs=3, max_q=64, seed=seed)
        reqs = []
        for r in arr:
            name = "ABC"[r.db]
            ct_all = ctA if name == "A" else ctB
            parts = [(i, i + 1) for i in range(r.Q)] if per_query else [(0, r.Q)]
            for a, b in parts:
                req = serve.Request(r.rid, name, ct_all[a:b], r.k, arrival=r.arrival_s)
                req.pool_rows = np.arange(a, b) % pool
                reqs.append(req)
        return reqs

    def distances_of(req):
        if req.db == "C":
            return req.Q * srv.n_clusters + srv.requested_pairs(req.selected)
        return req.Q * n_of[req.db]

    def serve_trace(reqs, max_batch, inflight, realtime):
        # buffers cached by the previous trace's server go back to the device
        # first (outside the timed region), so that one trace's pools cannot
        # push the caching allocator into a synchronising retry in the next
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
        s = serve.Server(dbs, hbm_budget=budget, max_inflight=inflight,
                         max_batch_queries=max_batch, client_select=select,
                         keep_outputs=False)
        t0 = time.perf_counter()
        done = s.run(reqs, realtime=realtime)
        wall = time.perf_counter() - t0
        # a request split into parts completes when its last part does
        by_rid = {}
        for r in done:
            a, dn = by_rid.get(r.rid, (r.arrival, r.done))
            by_rid[r.rid] = (min(a, r.arrival), max(dn, r.done))
        lat = np.array([1e3 * (dn - a) for a, dn in by_rid.values()])
        st = {"requests": len(by_rid), "p50_ms": round(pct(lat, 50), 3),
              "p99_ms": round(pct(lat, 99), 3), "mean_ms": round(float(lat.mean()), 3)}
        st["distances_per_s"] = round(sum(distances_of(r) for r in done) / wall, 1)
        st["wall_s"] = round(wall, 3)
        st["launches"] = s.launches
        st["peak_hbm_bytes"] = s.peak_used
        return st

    nreq = args.serving_requests
    # warm-up, then capacity: every request present at t = 0
    serve_trace(make_requests(1000.0, 20, synthdata.SEED_ARR + 50), 64, 3, False)
    cap = serve_trace(make_requests(1000.0, nreq, synthdata.SEED_ARR + 5), 64, 3, False)
    cap_rate = nreq / cap["wall_s"]
    log(f"serving capacity {cap_rate:.1f} req/s: {cap}")
    out = {"capacity_req_per_s": round(cap_rate, 2), "saturated": cap}
    for rho in (0.5, 0.9):
        st = serve_trace(make_requests(rho * cap_rate, nreq, synthdata.SEED_ARR + 5), 64, 3,
                         True)
        log(f"rho={rho}: {st}")
        out[f"rho_{rho}"] = st
    if args.serving_rate > 0:
        st = serve_trace(make_requests(args.serving_rate, nreq, synthdata.SEED_ARR + 5), 64, 3,
                         True)
        log(f"rate {args.serving_rate} req/s: {st}")
        out[f"rate_{args.serving_rate}"] = st
    # the per-query path: one query per launch, one launch at a time
    per_q = serve_trace(make_requests(1000.0, max(10, nreq // 10), synthdata.SEED_ARR + 5,
                                      per_query=True), 1, 1, False)
    log(f"per-query path (saturated): {per_q}")
    out["per_query_path_saturated"] = per_q
    return {
        "metric": "serving: p50/p99 arrival-to-shares latency and encrypted distances/s",
        "value": out["rho_0.9"]["distances_per_s"], "unit": UNIT, "n_gpus": 1,
        "steps": nreq, "warmup": 20, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u64", "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals, Q ~ U{1..64}, k in {1,10,100}, "
                               "databases 100K x 128 uint8, 1M x 96 int8, clustered 10M x 96 "
                               "int8 (64 clusters per query); fused batched launches, "
                               "3 in flight, <= 64 queries per launch",
                   "hbm_budget_gib": round(budget / (1 << 30), 1)},
        "latency": {"p50_ms_rho_0.9": out["rho_0.9"]["p50_ms"],
                    "p99_ms_rho_0.9": out["rho_0.9"]["p99_ms"],
                    "p50_ms_rho_0.5": out["rho_0.5"]["p50_ms"],
                    "p99_ms_rho_0.5": out["rho_0.5"]["p99_ms"]},
        "serving": out,
        "batched_vs_per_query": round(cap["distances_per_s"] / per_q["distances_per_s"], 2),
    }


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
                          "frac": round(mac1_gbs / HBM_PEAK_GBS, 4),
                          "traffic": recorded_traffic("k_mac",
                                                      "fused_1Mx128_q1_hbm_counters.md"),
                          "traffic_unit": "bytes/launch",
                          "avg_ms": round(fph["mac"], 4),
                          "algorithmic": f"{mac1_bytes} B (resident DB + query NTT "
                                         "read + NTT-form outputs written)",
                          "bytes_per_distance": round(mac1_bytes / n, 1),
                          "modular_mul_acc_per_s": round(2 * d * L * N * C /
                                                         (fph["mac"] * 1e-3), 1),
                          "distances_per_s_in_kernel": round(n / (fph["mac"] * 1e-3), 1)}}
    log(f"fused Q=1: p50 {fused['query_p50_ms']} ms, {fused_value / 1e9:.3f} G/s, "
        f"mac {mac1_gbs:.0f} GB/s")
    return fused


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def host_threads() -> int:
    """Threads this process may run the oracle on: its CPU affinity, capped
    by OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        n = min(n, int(env))
    return max(1, n)


def _oracle_chunk_inputs(oracle, w, pts, slot, qv, N, L, t, k=0):
    P = oracle.Params(N, oracle.rns_primes(N, L), t)
    assert P.t == t
    d = pts.shape[1]
    s = synthdata.gen_secret(N, 1)
    a = synthdata.gen_uniform_a(P.qs, N, d, 2)
    e = synthdata.gen_cbd_error(N, d, 2)
    ct = oracle.encrypt_constants(P, s, a, e, [int(x) for x in qv])
    return P, ct


def cpu_baseline(w, pts, slot, qv, N, L, t):
    """The oracle, as it stands, on this host's cores (its client encryption
    is done first and not timed; the server stage -- schoolbook negacyclic
    products for 2 components x L limbs x d coordinates, masks and the norm
    plaintext -- is):
      * all cores: one chunk (N slots) of this database for one query; the
        workload's rate is N / that time (extrapolated from one of its chunks);
      * one thread: the same chunk's output at 256 of its N coefficient
        positions (the oracle's per-coefficient routine), extrapolated to N;
      * the 10,000 x 128 uint8 linear scan (N = 4096, L = 2, 3 chunks) in
        full, on all cores and (one chunk, extrapolated x3) on one thread."""
    import oracle
    threads = oracle.set_threads(host_threads())
    key = synthdata.gen_mask_key(3)
    d = pts.shape[1]
    P, ct = _oracle_chunk_inputs(oracle, w, pts, slot, qv, N, L, t)
    g, nrm = oracle.chunk_plaintexts(pts, slot, N, 0)
    t0 = time.perf_counter()
    oracle.server_chunk(P, ct, g, nrm, key, 0, 0)
    dt_all = time.perf_counter() - t0
    oracle.set_threads(1)
    js = list(range(0, N, N // 256))
    t0 = time.perf_counter()
    oracle.server_coeffs(P, ct, g, nrm, key, 0, 0, js)
    dt_one = (time.perf_counter() - t0) * N / len(js)
    log(f"cpu oracle ({cpu_model()}): one chunk {dt_all:.2f}s on {threads} threads, "
        f"{dt_one:.1f}s on one thread (extrapolated)")
    # the 10,000 x 128 workload in full
    w1 = synthdata.WORKLOADS[1]
    p1 = synthdata.gen_points(w1)
    q1 = synthdata.gen_queries(w1, 1)[0]
    t1 = oracle.plain_modulus(w1.N, w1.t_bits)
    s1 = synthdata.gen_slot_map(len(p1), w1.N, synthdata.SEED_PERM + 1)
    P1, ct1 = _oracle_chunk_inputs(oracle, w1, p1, s1, q1, w1.N, w1.L, t1)
    C1 = len(s1) // w1.N
    chunks = [oracle.chunk_plaintexts(p1, s1, w1.N, k) for k in range(C1)]
    oracle.set_threads(threads)
    t0 = time.perf_counter()
    for k, (gk, nk) in enumerate(chunks):
        oracle.server_chunk(P1, ct1, gk, nk, key, 0, k)
    dt1_all = time.perf_counter() - t0
    oracle.set_threads(1)
    t0 = time.perf_counter()
    oracle.server_chunk(P1, ct1, chunks[0][0], chunks[0][1], key, 0, 0)
    dt1_one = (time.perf_counter() - t0) * C1
    oracle.set_threads(threads)
    log(f"cpu oracle, 10K x 128 in full: {dt1_all:.2f}s on {threads} threads, "
        f"{dt1_one:.1f}s on one thread (one chunk x {C1})")
    return {"value": round(N / dt_all, 1), "unit": UNIT, "cores": threads, "kind": "oracle",
            "sample": f"one chunk ({N} slots) of the {len(pts):,} x {d} database, one query, "
                      f"on {threads} threads: schoolbook negacyclic products for 2 components "
                      f"x {L} limbs x {d} coordinates, masks and norm plaintext (encryption "
                      f"not timed); extrapolated to the database: N / chunk time",
            "extrapolated": True, "seconds": round(dt_all, 2),
            "cpu_model": cpu_model(),
            "single_thread": {"value": round(N / dt_one, 1), "unit": UNIT, "cores": 1,
                              "sample": f"the same chunk at {len(js)} of its {N} coefficient "
                                        "positions, extrapolated to N",
                              "extrapolated": True, "seconds_per_chunk": round(dt_one, 2)},
            "workload_10Kx128_full": {
                "distances": len(p1), "chunks": C1, "N": w1.N, "L": w1.L,
                "all_cores": {"value": round(len(p1) / dt1_all, 1), "unit": UNIT,
                              "cores": threads, "seconds": round(dt1_all, 2),
                              "extrapolated": False},
                "single_thread": {"value": round(len(p1) / dt1_one, 1), "unit": UNIT,
                                  "cores": 1, "seconds": round(dt1_one, 2),
                                  "extrapolated": True,
                                  "sample": f"one of its {C1} chunks, times {C1}"}}}


if __name__ == "__main__":
    main()
